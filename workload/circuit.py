"""Syndrome-extraction circuits with circuit-level noise, as a flat op list.

This module only builds the *workload*: which gate, noise location,
initialisation or measurement happens in which order (Sec. III, Fig. 1).  It
holds none of the simulation arithmetic; both the oracle and the GPU engine
consume the same op list as input data.

Circuit (memory experiment, Sec. III): data start in |0>, then C rounds.  A
round is an X-phase followed by a Z-phase.  A phase is one init tick (the P
ancillas of that type, X-ancillas in |+>, Z-ancillas in |0>), T CNOT ticks and
one measure tick.  X-phase CNOTs go ancilla -> data and the ancilla is
measured in X; Z-phase CNOTs go data -> ancilla and the ancilla is measured in
Z.  After the last round every data qubit is measured in Z, which fixes the
logical Z (the parity of all data bits, since Z-bar = Z^n for odd n).

The paper's optimised schedule (its ref. on colour-code decoding) is not
available, so the T CNOT layers are a proper edge colouring of the
face/data incidence graph (T = max degree: 4 at d=3, 6 at d>=5).  All CNOTs of
one phase commute, so any proper colouring measures the checks.

Noise placement (Fig. 1b-d): one single-qubit error location after every
CNOT on each of its two qubits, one on every live qubit that is idle in a
CNOT tick, and one after every initialisation or reset.  Measurements are
noiseless (Sec. III.A).  Within a tick all gates come first and then the
noise ops of every live qubit in ascending leaf order.  The CNOTs of a tick are
listed in a centre-walk order (`_CentreWalk`), which changes no result.

Channels per location: "srx" (Eq. 1), "ad" (Eq. 2-3), "srx+ad" (SRX then AD
at the same location, one theta and one gamma), and their Pauli-twirled twins
"pta_srx", "pta_ad", "pta_srx+ad" (Eq. 9), or "none".
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .colorcode import ColorCode, build_color_code

# op codes
OP_INIT, OP_CNOT, OP_SRX, OP_AD, OP_PAULI, OP_MEAS = 0, 1, 2, 3, 4, 5
OP_NAMES = {OP_INIT: "init", OP_CNOT: "cnot", OP_SRX: "srx", OP_AD: "ad",
            OP_PAULI: "pauli", OP_MEAS: "meas"}
# op-list columns
C_OP, C_Q0, C_Q1, C_ARG, C_LOC, C_DRAW, C_REC, C_PREV, C_TICK = range(9)
N_COLS = 9

CHANNELS = ("none", "srx", "ad", "srx+ad", "pta_srx", "pta_ad", "pta_srx+ad")


@dataclass
class Circuit:
    code: ColorCode
    rounds: int
    channel: str
    n_qubits: int
    n_leaves: int
    leaf_of_qubit: np.ndarray     # [n_qubits] int32
    ops: np.ndarray               # [n_ops, N_COLS] int32
    n_loc: int                    # noise locations (theta/gamma index range)
    n_draws: int                  # random draws per trajectory
    n_rec: int                    # measurement record bits per trajectory
    n_ad: int                     # AD ops (Kraus branch bits) per trajectory
    ad_ops: np.ndarray            # op indices of AD ops, in order
    data_rec: np.ndarray          # [n] record index of data qubit k's final bit
    xsyn_rec: np.ndarray          # [rounds, P] record index of X-check p in round r
    zsyn_rec: np.ndarray          # [rounds, P]
    ticks: int

    @property
    def n_ops(self) -> int:
        return int(self.ops.shape[0])

    def count(self, op: int) -> int:
        return int((self.ops[:, C_OP] == op).sum())


def edge_colouring(checks: np.ndarray) -> np.ndarray:
    """Proper edge colouring of the bipartite face/data graph with max-degree
    colours (Koenig), by alternating-path recolouring.  Returns colour[f, k]
    (-1 where there is no edge)."""
    P, n = checks.shape
    deg = max(int(checks.sum(1).max()), int(checks.sum(0).max()))
    col = -np.ones((P, n), dtype=np.int64)
    at_f = [dict() for _ in range(P)]   # colour -> data k
    at_q = [dict() for _ in range(n)]   # colour -> face f
    for f in range(P):
        for k in range(n):
            if not checks[f, k]:
                continue
            a = next(c for c in range(deg) if c not in at_f[f])
            b = next(c for c in range(deg) if c not in at_q[k])
            if a not in at_q[k]:
                c = a
            else:
                # swap a/b along the alternating path that starts at data k
                # with an a-edge; it cannot reach face f (bipartite argument)
                path = []
                side, v, want = "q", k, a
                while True:
                    table = at_q[v] if side == "q" else at_f[v]
                    if want not in table:
                        break
                    w = table[want]
                    path.append((w, v, want) if side == "q" else (v, w, want))
                    side = "f" if side == "q" else "q"
                    v = w
                    want = b if want == a else a
                for (ff, kk, cc) in path:
                    del at_f[ff][cc]
                    del at_q[kk][cc]
                for (ff, kk, cc) in path:
                    nc = b if cc == a else a
                    at_f[ff][nc] = kk
                    at_q[kk][nc] = ff
                    col[ff, kk] = nc
                c = a
            col[f, k] = c
            at_f[f][c] = k
            at_q[k][c] = f
    return col


class _CentreWalk:
    """Order of the CNOTs inside one tick.

    The CNOTs of a tick act on disjoint qubits, so every order gives the same
    circuit.  A tree-tensor-network simulator in canonical form brings its
    orthogonality centre to one end of every CNOT, and to the qubit of every
    measurement and amplitude-damping jump (Sec. III.B); the remaining order
    only decides how far that centre travels.  This walk models it on the
    binary tree (bottom node of qubit q = L/2 + leaf(q)/2, heap numbering,
    root 1): the next CNOT is the one whose nearer end is closest to the
    current position (ties by the leaf-sorted order), and the centre then
    rests at that end.  It changes no amplitude, probability or draw; it
    only shortens the path, by about 15% of the centre moves of the d=5
    circuits."""

    def __init__(self, leaf_of_qubit: np.ndarray, n_leaves: int):
        self.leaf = leaf_of_qubit
        self.half = n_leaves // 2
        self.at = 1

    def node(self, q: int) -> int:
        return self.half + int(self.leaf[q]) // 2

    @staticmethod
    def dist(a: int, b: int) -> int:
        n = 0
        while a != b:
            if a > b:
                a //= 2
            else:
                b //= 2
            n += 1
        return n

    def _end(self, c: int, t: int):
        nc, nt = self.node(c), self.node(t)
        if nc == nt:
            return 0, self.at
        dc, dt = self.dist(self.at, nc), self.dist(self.at, nt)
        return (dc, nc) if dc <= dt else (dt, nt)

    def order(self, gates):
        pend = list(gates)
        out = []
        at = self.at
        while pend:
            best = min(range(len(pend)), key=lambda i: (self._end(*pend[i])[0], i))
            g = pend.pop(best)
            out.append(g)
            self.at = self._end(*g)[1]
        self.at = at            # visit() moves it as the gates are emitted
        return out

    def visit(self, op: int, q0: int, q1: int):
        if op == OP_CNOT:
            self.at = self._end(q0, q1)[1]
        elif op in (OP_MEAS, OP_AD):
            self.at = self.node(q0)


def default_layout(code: ColorCode) -> np.ndarray:
    """Qubit i on leaf i (the paper's default ordering, App. B)."""
    return np.arange(code.n_qubits, dtype=np.int32)


def snake_layout(code: ColorCode) -> np.ndarray:
    """The snake ordering of App. B (Fig. 8a, Table III): a path through the
    lattice that runs along each row of points and turns back at its end,
    so consecutive rows are swept in opposite directions (a face centre
    contributes its X- and then its Z-ancilla); qubit number k on the path
    goes to leaf k.  The figure's path is not reproduced in the text; this is
    the boustrophedon of the same row sweep that defines the default labels."""
    m = 3 * (code.d - 1) // 2
    at = {}
    for lab in sorted(code.coords):
        at.setdefault(tuple(code.coords[lab]), []).append(lab)
    path = []
    for j in range(m + 1):
        row = [(i, j) for i in range(m + 1 - j)]
        if j % 2 == 1:
            row.reverse()
        for pt in row:
            path += at[pt]
    leaf = np.empty(code.n_qubits, dtype=np.int32)
    leaf[np.asarray(path)] = np.arange(len(path), dtype=np.int32)
    return leaf


def n_leaves_for(n_qubits: int) -> int:
    L = 2
    while L < n_qubits:
        L *= 2
    return L


def build_circuit(d: int, rounds: int, channel: str,
                  leaf_of_qubit: np.ndarray | str | None = None) -> Circuit:
    """leaf_of_qubit: an explicit qubit -> leaf map, "default" / None (qubit i
    on leaf i), "snake" (App. B, Fig. 8a), or "optimized" (App. B,
    Algorithm 1: best of 8 clustered layouts by the exact bond dimension of
    the circuit's Clifford skeleton)."""
    if channel not in CHANNELS:
        raise ValueError(f"unknown channel {channel!r}")
    if rounds < 1:
        raise ValueError("rounds must be >= 1")
    code = build_color_code(d)
    N = code.n_qubits
    if isinstance(leaf_of_qubit, str) and leaf_of_qubit == "optimized":
        from .layout import optimized_layout
        skeleton = build_circuit(d, rounds, "none")
        leaf_of_qubit, _ = optimized_layout(skeleton.ops, N)
    elif leaf_of_qubit is None or (isinstance(leaf_of_qubit, str) and leaf_of_qubit == "default"):
        leaf_of_qubit = default_layout(code)
    elif isinstance(leaf_of_qubit, str) and leaf_of_qubit == "snake":
        leaf_of_qubit = snake_layout(code)
    leaf_of_qubit = np.asarray(leaf_of_qubit, dtype=np.int32)
    L = n_leaves_for(N)
    if sorted(leaf_of_qubit.tolist()) != sorted(set(leaf_of_qubit.tolist())) or \
            leaf_of_qubit.min() < 0 or leaf_of_qubit.max() >= L:
        raise ValueError("leaf_of_qubit must be an injective map into [0, L)")
    colouring = edge_colouring(code.checks)
    T = int(colouring.max()) + 1
    P, n = code.n_plaq, code.n

    def by_leaf(qs):
        return sorted(qs, key=lambda q: int(leaf_of_qubit[q]))

    rows = []
    state = {"loc": 0, "draw": 0, "rec": 0, "tick": 0}
    last_meas = {}   # qubit -> (basis, record index)
    walk = _CentreWalk(leaf_of_qubit, L)

    def emit(op, q0, q1=-1, arg=0, loc=-1, draw=-1, rec=-1, prev=-1):
        rows.append((op, q0, q1, arg, loc, draw, rec, prev, state["tick"]))
        walk.visit(op, q0, q1)

    def noise(q):
        loc = state["loc"]
        state["loc"] += 1
        parts = {"none": (), "srx": ("srx",), "ad": ("ad",), "srx+ad": ("srx", "ad"),
                 "pta_srx": ("psrx",), "pta_ad": ("pad",),
                 "pta_srx+ad": ("psrx", "pad")}[channel]
        for p in parts:
            if p == "srx":
                emit(OP_SRX, q, loc=loc)
            elif p == "ad":
                emit(OP_AD, q, loc=loc, draw=state["draw"])
                state["draw"] += 1
            else:
                emit(OP_PAULI, q, arg=0 if p == "psrx" else 1, loc=loc,
                     draw=state["draw"])
                state["draw"] += 1

    def init_tick(qs, basis):
        for q in by_leaf(qs):
            pb, pr = last_meas.get(q, (-1, -1))
            emit(OP_INIT, q, arg=basis, rec=pr, prev=pb)
        for q in by_leaf(qs):
            noise(q)
        state["tick"] += 1

    def meas(q, basis):
        r = state["rec"]
        emit(OP_MEAS, q, arg=basis, rec=r, draw=state["draw"])
        state["rec"] += 1
        state["draw"] += 1
        last_meas[q] = (basis, r)
        return r

    data_q = [int(x) for x in code.data_label]
    xsyn = np.zeros((rounds, P), dtype=np.int64)
    zsyn = np.zeros((rounds, P), dtype=np.int64)
    init_tick(data_q, 0)
    for r in range(rounds):
        for phase in ("X", "Z"):
            anc = code.xanc_label if phase == "X" else code.zanc_label
            anc_q = [int(x) for x in anc]
            init_tick(anc_q, 1 if phase == "X" else 0)
            live = data_q + anc_q
            for t in range(T):
                gates = []
                for f in range(P):
                    for k in range(n):
                        if colouring[f, k] == t:
                            a, dq = int(anc[f]), int(code.data_label[k])
                            gates.append((a, dq) if phase == "X" else (dq, a))
                gates.sort(key=lambda g: (int(leaf_of_qubit[g[0]]), int(leaf_of_qubit[g[1]])))
                for c_, t_ in walk.order(gates):
                    emit(OP_CNOT, c_, t_)
                for q in by_leaf(live):
                    noise(q)
                state["tick"] += 1
            order = sorted(range(P), key=lambda f: int(leaf_of_qubit[anc[f]]))
            for f in order:
                rr = meas(int(anc[f]), 1 if phase == "X" else 0)
                (xsyn if phase == "X" else zsyn)[r, f] = rr
            state["tick"] += 1
    data_rec = np.zeros(n, dtype=np.int64)
    for k in sorted(range(n), key=lambda k: int(leaf_of_qubit[code.data_label[k]])):
        data_rec[k] = meas(int(code.data_label[k]), 0)
    state["tick"] += 1
    ops = np.asarray(rows, dtype=np.int32).reshape(-1, N_COLS)
    ad_ops = np.nonzero(ops[:, C_OP] == OP_AD)[0].astype(np.int64)
    return Circuit(code=code, rounds=rounds, channel=channel, n_qubits=N,
                   n_leaves=L, leaf_of_qubit=leaf_of_qubit, ops=ops,
                   n_loc=state["loc"], n_draws=state["draw"], n_rec=state["rec"],
                   n_ad=len(ad_ops), ad_ops=ad_ops, data_rec=data_rec,
                   xsyn_rec=xsyn, zsyn_rec=zsyn, ticks=state["tick"])


def ops_per_shot(circ: Circuit) -> int:
    """Every state-touching op: CNOTs, noise ops, inits/resets, measurements."""
    return circ.n_ops


def uniform_params(circ: Circuit, rows: int, theta=None, gamma=None) -> tuple:
    """Per-trajectory, per-location noise parameters as [rows, n_loc] float64.
    `theta`/`gamma` may be a scalar or a per-row array."""
    th = np.zeros((rows, circ.n_loc))
    ga = np.zeros((rows, circ.n_loc))
    if theta is not None:
        th[:] = np.asarray(theta, dtype=np.float64).reshape(-1, 1) if np.ndim(theta) else theta
    if gamma is not None:
        ga[:] = np.asarray(gamma, dtype=np.float64).reshape(-1, 1) if np.ndim(gamma) else gamma
    return th, ga


class _Stub:
    pass


def custom_circuit(n_qubits: int, program, data_qubits=None, leaf_of_qubit=None) -> Circuit:
    """Build an op list from a small program, for tests and examples.

    program: sequence of tuples
      ("init", q, basis)   basis 0 -> |0>, 1 -> |+> (reset from its last outcome)
      ("cnot", c, t)       ("srx", q)   ("ad", q)   ("srxad", q)
      ("pauli", q, kind)   kind 0 -> twirled SRX, 1 -> twirled AD
      ("meas", q, basis)   basis 0 -> Z, 1 -> X
      ("tick",)            closes the current tick
    Every noise op gets its own location index.  `data_qubits` are live from
    the start in |0> (default: all qubits)."""
    if data_qubits is None:
        data_qubits = list(range(n_qubits))
    if leaf_of_qubit is None:
        leaf_of_qubit = np.arange(n_qubits, dtype=np.int32)
    rows = []
    loc = draw = rec = tick = 0
    last = {}
    data_rec = {}
    for ins in program:
        kind = ins[0]
        if kind == "tick":
            tick += 1
            continue
        q = int(ins[1])
        if kind == "init":
            pb, pr = last.get(q, (-1, -1))
            rows.append((OP_INIT, q, -1, int(ins[2]), -1, -1, pr, pb, tick))
        elif kind == "cnot":
            rows.append((OP_CNOT, q, int(ins[2]), 0, -1, -1, -1, -1, tick))
        elif kind == "srx":
            rows.append((OP_SRX, q, -1, 0, loc, -1, -1, -1, tick))
            loc += 1
        elif kind == "ad":
            rows.append((OP_AD, q, -1, 0, loc, draw, -1, -1, tick))
            loc += 1
            draw += 1
        elif kind == "srxad":
            rows.append((OP_SRX, q, -1, 0, loc, -1, -1, -1, tick))
            rows.append((OP_AD, q, -1, 0, loc, draw, -1, -1, tick))
            loc += 1
            draw += 1
        elif kind == "pauli":
            rows.append((OP_PAULI, q, -1, int(ins[2]), loc, draw, -1, -1, tick))
            loc += 1
            draw += 1
        elif kind == "meas":
            b = int(ins[2])
            rows.append((OP_MEAS, q, -1, b, -1, draw, rec, -1, tick))
            last[q] = (b, rec)
            data_rec[q] = rec
            rec += 1
            draw += 1
        else:
            raise ValueError(kind)
    ops = np.asarray(rows, dtype=np.int32).reshape(-1, N_COLS)
    code = _Stub()
    code.data_label = np.asarray(data_qubits, dtype=np.int64)
    code.n = len(data_qubits)
    code.n_plaq = 0
    code.checks = np.zeros((0, len(data_qubits)), dtype=np.uint8)
    ad_ops = np.nonzero(ops[:, C_OP] == OP_AD)[0].astype(np.int64) if len(rows) else np.zeros(0, np.int64)
    drec = np.array([data_rec.get(int(q), -1) for q in data_qubits], dtype=np.int64)
    return Circuit(code=code, rounds=0, channel="custom", n_qubits=n_qubits,
                   n_leaves=n_leaves_for(n_qubits), leaf_of_qubit=np.asarray(leaf_of_qubit, dtype=np.int32),
                   ops=ops, n_loc=loc, n_draws=draw, n_rec=rec, n_ad=len(ad_ops), ad_ops=ad_ops,
                   data_rec=drec, xsyn_rec=np.zeros((0, 0), np.int64),
                   zsyn_rec=np.zeros((0, 0), np.int64), ticks=tick + 1)


def random_program(n_qubits: int, depth: int, rng: np.random.Generator,
                   noise=("srx",), measure_every: int = 0, p_twoq: float = 0.6):
    """A random circuit over n qubits: random CNOTs (any pair), noise ops and
    optional mid-circuit measure+re-init of random qubits; ends with a Z
    measurement of every qubit.  Returns a program for `custom_circuit`."""
    prog = [("init", q, int(rng.integers(0, 2))) for q in range(n_qubits)]
    prog.append(("tick",))
    for layer in range(depth):
        if rng.random() < p_twoq or n_qubits < 2:
            for _ in range(max(1, n_qubits // 3)):
                if n_qubits >= 2:
                    c, t = rng.choice(n_qubits, size=2, replace=False)
                    prog.append(("cnot", int(c), int(t)))
        for q in range(n_qubits):
            kind = noise[int(rng.integers(0, len(noise)))]
            if kind == "pauli_srx":
                prog.append(("pauli", q, 0))
            elif kind == "pauli_ad":
                prog.append(("pauli", q, 1))
            else:
                prog.append((kind, q))
        if measure_every and (layer + 1) % measure_every == 0:
            q = int(rng.integers(0, n_qubits))
            b = int(rng.integers(0, 2))
            prog.append(("meas", q, b))
            prog.append(("init", q, int(rng.integers(0, 2))))
        prog.append(("tick",))
    for q in range(n_qubits):
        prog.append(("meas", q, 0))
    return prog
