"""The colour-code workload: code parameters fixed by the paper (Sec. II.A,
App. A.1) and the circuit structure of Sec. III / Fig. 1."""
import itertools

import numpy as np
import pytest

from workload import (build_color_code, build_circuit, gf2_rank, edge_colouring,
                      OP_CNOT, OP_INIT, OP_MEAS, OP_SRX, OP_AD, OP_PAULI,
                      C_OP, C_Q0, C_Q1, C_TICK, C_LOC, C_DRAW, C_REC)


@pytest.mark.parametrize("d,n,P,N", [(3, 7, 3, 13), (5, 19, 9, 37), (7, 37, 18, 73)])
def test_code_counts(d, n, P, N):
    # [[(3d^2+1)/4, 1, d]] and two ancillas per plaquette (Sec. II.A)
    c = build_color_code(d)
    assert c.n == n == (3 * d * d + 1) // 4
    assert c.n_plaq == P
    assert c.n_qubits == N
    w = c.checks.sum(1)
    assert set(w.tolist()) <= {4, 6}             # weight 4 on the boundary, 6 in the bulk
    assert (c.checks.sum(0) <= 3).all()
    # X and Z checks on the same supports commute iff every overlap is even
    assert not ((c.checks.astype(int) @ c.checks.T.astype(int)) % 2).any()
    # k = n - rank(H_X) - rank(H_Z) = 1
    assert c.n - 2 * gf2_rank(c.checks) == 1
    # three-colourable faces: touching faces differ in colour
    for a, b in itertools.combinations(range(P), 2):
        if (c.checks[a] & c.checks[b]).any():
            assert c.colour[a] != c.colour[b]


def _min_logical_weight(checks, max_w):
    n = checks.shape[1]
    rank = gf2_rank(checks)
    for w in range(1, max_w + 1):
        for sup in itertools.combinations(range(n), w):
            v = np.zeros(n, dtype=np.uint8)
            v[list(sup)] = 1
            if ((checks.astype(int) @ v) % 2).any():
                continue
            # commutes with every check; logical iff not in the check row space
            if gf2_rank(np.vstack([checks, v])) > rank:
                return w
    return None


@pytest.mark.parametrize("d", [3, 5])
def test_code_distance(d):
    c = build_color_code(d)
    assert _min_logical_weight(c.checks, d) == d


@pytest.mark.parametrize("d,C,ch,ops,cnot,loc", [
    (3, 1, "srx", 143, 24, 93), (3, 3, "ad", 387, 72, 265),
    (5, 5, "srx", 2427, 420, 1789), (5, 3, "srx+ad", 2560, 252, 1081)])
def test_op_counts(d, C, ch, ops, cnot, loc):
    circ = build_circuit(d, C, ch)
    c = circ.code
    T = 4 if d == 3 else 6
    n, P = c.n, c.n_plaq
    assert circ.n_loc == 2 * C * (T * (n + P) + P) + n == loc
    assert circ.count(OP_CNOT) == 2 * C * int(c.checks.sum()) == cnot
    assert circ.count(OP_INIT) == circ.count(OP_MEAS) == 2 * P * C + n
    assert circ.n_ops == ops
    assert circ.n_rec == 2 * P * C + n


def test_schedule_is_proper_and_complete():
    for d in (3, 5, 7):
        circ = build_circuit(d, 2, "srx")
        ops = circ.ops
        for t in np.unique(ops[:, C_TICK]):
            sel = ops[(ops[:, C_TICK] == t) & (ops[:, C_OP] == OP_CNOT)]
            qs = np.concatenate([sel[:, C_Q0], sel[:, C_Q1]])
            assert len(qs) == len(set(qs.tolist()))          # one gate per qubit per tick
        # every face/data edge appears once per phase, in both phases of every round
        c = circ.code
        cn = ops[ops[:, C_OP] == OP_CNOT]
        assert len(cn) == 2 * circ.rounds * int(c.checks.sum())
        col = edge_colouring(c.checks)
        assert col.max() + 1 == (4 if d == 3 else 6)


def test_noise_every_live_qubit_every_cnot_tick():
    circ = build_circuit(5, 1, "srx")
    ops = circ.ops
    c = circ.code
    for t in np.unique(ops[:, C_TICK]):
        sel = ops[ops[:, C_TICK] == t]
        if (sel[:, C_OP] == OP_CNOT).any():
            noisy = sel[sel[:, C_OP] == OP_SRX][:, C_Q0]
            assert len(noisy) == c.n + c.n_plaq == len(set(noisy.tolist()))
        if (sel[:, C_OP] == OP_MEAS).any():
            assert not (sel[:, C_OP] == OP_SRX).any()       # measurements are noiseless


def test_indices_dense():
    circ = build_circuit(3, 3, "srx+ad")
    ops = circ.ops
    locs = ops[ops[:, C_LOC] >= 0][:, C_LOC]
    assert set(locs.tolist()) == set(range(circ.n_loc))
    draws = ops[ops[:, C_DRAW] >= 0][:, C_DRAW]
    assert sorted(draws.tolist()) == list(range(circ.n_draws))
    recs = ops[ops[:, C_OP] == OP_MEAS][:, C_REC]
    assert sorted(recs.tolist()) == list(range(circ.n_rec))
    assert circ.n_ad == circ.count(OP_AD) == circ.n_loc


# ------------------------------------------------------------------ layout ----
def test_layout_exact_bond_dims_match_table_iii():
    # App. B, Table III (C = 1): d=3 default 8 / optimized 8; d=5 default 512 /
    # optimized 16 (the Clifford skeleton already needs the tabulated values)
    from workload import exact_bond_dim, optimized_layout
    for d, want_def, want_opt in ((3, 8, 8), (5, 512, 16)):
        circ = build_circuit(d, 1, "none")
        assert exact_bond_dim(circ.ops, circ.n_qubits, circ.leaf_of_qubit) == want_def
        lay, chi = optimized_layout(circ.ops, circ.n_qubits)
        assert chi <= want_opt
        assert sorted(set(lay.tolist())) == sorted(lay.tolist())
        assert lay.min() >= 0 and lay.max() < circ.n_leaves
        assert exact_bond_dim(circ.ops, circ.n_qubits, lay) == chi


def test_layout_exact_bond_dim_matches_oracle_stabilizer_ranks():
    # the compile-time scorer against the oracle's tableau + Schmidt ranks,
    # on random layouts, over every op of the circuit
    from workload import exact_bond_dim
    from oracle import chp, stabrank
    g = np.random.default_rng(3)
    for trial in range(3):
        circ0 = build_circuit(3, 1, "none")
        lay = g.permutation(circ0.n_leaves)[:circ0.n_qubits].astype(np.int32)
        circ = build_circuit(3, 1, "none", leaf_of_qubit=lay)
        best = 1
        for k in range(circ.n_ops):
            _, tab = chp.run(circ, 0.0, 0.0, 0, np.arange(1), stop_after_op=k)
            r = stabrank.tree_bond_ranks(tab.stabilizers(), circ.leaf_of_qubit, circ.n_leaves)
            best = max(best, max(r.values()))
        assert exact_bond_dim(circ.ops, circ.n_qubits, circ.leaf_of_qubit) == best


def test_optimized_layout_keeps_the_circuit():
    # the layout moves qubits between leaves; the op list is the same circuit
    a = build_circuit(5, 2, "srx")
    b = build_circuit(5, 2, "srx", leaf_of_qubit="optimized")
    assert a.n_ops == b.n_ops and a.n_loc == b.n_loc and a.n_rec == b.n_rec
    key = lambda ops: sorted(map(tuple, ops[:, [0, 1, 2, 3, 8]].tolist()))
    assert key(a.ops) == key(b.ops)


def test_snake_layout_is_a_path_through_the_lattice():
    # App. B (Fig. 8a): consecutive qubits of the snake sit on the same or
    # neighbouring lattice points, and the map is a bijection onto leaves 0..N-1
    from workload import build_color_code, snake_layout
    nb = {(1, 0), (-1, 0), (0, 1), (0, -1), (1, -1), (-1, 1), (0, 0)}
    for d in (3, 5, 7):
        c = build_color_code(d)
        leaf = snake_layout(c)
        assert sorted(leaf.tolist()) == list(range(c.n_qubits))
        order = np.argsort(leaf)
        for a, b in zip(order[:-1], order[1:]):
            pa, pb = c.coords[int(a)], c.coords[int(b)]
            assert (pb[0] - pa[0], pb[1] - pa[1]) in nb, (d, a, b, pa, pb)


# Exact bond dimension of the Clifford skeleton (gates, resets and
# measurements without noise) for the three orderings of App. B, Table III,
# on this build's schedule: (d, C) -> (default, snake, optimized).  The paper's
# AD values are d3C1 8/8/8 and d5C1 512/256/16 (C=1 columns reproduced
# except the d=5 snake, whose path the text does not give); at C = d the
# paper's AD runs grow further (d3C3 32/16/16, d5C5 2048/1024/256) because
# damping leaves the stabilizer states that the skeleton keeps; d7C1: paper
# >=2048/2048/256.
TABLE_III_SKELETON = {(3, 1): (8, 8, 8), (3, 3): (16, 8, 8), (5, 1): (512, 512, 16), (5, 5): (512, 512, 16),
                      (7, 1): (4096, 4096, 512)}


@pytest.mark.parametrize("d,C", sorted(TABLE_III_SKELETON))
def test_table3_orderings_exact_bond_dimension(d, C):
    from workload import exact_bond_dim, optimized_layout
    want = TABLE_III_SKELETON[(d, C)]
    got = []
    for lay in ("default", "snake"):
        sk = build_circuit(d, C, "none", leaf_of_qubit=lay)
        got.append(exact_bond_dim(sk.ops, sk.n_qubits, sk.leaf_of_qubit))
    sk = build_circuit(d, C, "none")
    got.append(optimized_layout(sk.ops, sk.n_qubits)[1])
    assert tuple(got) == want
    assert got[2] <= got[1] <= got[0]
