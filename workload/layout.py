"""Qubit-to-leaf layouts for the binary tree (App. B, Algorithm 1, Table III).

The tree is built from the root down: the qubits of a subtree are split into
two groups, one per child subtree, by spectral clustering on the similarity
f_qc(q_i, q_j) = |G(q_i) & G(q_j)| + 1 / (|G(q_i)| + |G(q_j)|) (Eq. B1, G(q) the
two-qubit gates acting on q).  If the two clusters do not fit the children's
capacity (2^(layer-1) leaves each), more clusters are tried and agglomerated
into two balanced groups; if no number of clusters gives a valid split the
qubits are split evenly at random.  Several candidate layouts are drawn and
the one with the smallest exact bond dimension is kept.

Candidates are scored by the exact bond dimension of the circuit's Clifford
skeleton (its gates, resets and measurements without noise): the largest
Schmidt rank 2^S over every tree bond and every time, S computed from the
stabilizer generators (S_A = rank of the generators restricted to A minus
|A|).  This is host-side compilation of the input; it holds nothing of the
trajectory simulation.
"""
from __future__ import annotations

import numpy as np

from .circuit import OP_CNOT, OP_INIT, OP_MEAS, C_OP, C_Q0, C_Q1, C_ARG, n_leaves_for


# ----------------------------------------------------------- similarity ----
def similarity_matrix(ops: np.ndarray, n_qubits: int) -> np.ndarray:
    """f_qc of Eq. B1 for every qubit pair (zero on the diagonal)."""
    ops = np.asarray(ops)
    cn = ops[ops[:, C_OP] == OP_CNOT]
    pair = np.zeros((n_qubits, n_qubits))
    for c, t in zip(cn[:, C_Q0], cn[:, C_Q1]):
        pair[c, t] += 1
        pair[t, c] += 1
    deg = pair.sum(axis=1)
    with np.errstate(divide="ignore"):
        inv = 1.0 / (deg[:, None] + deg[None, :])
    inv[~np.isfinite(inv)] = 0.0
    W = pair + inv
    np.fill_diagonal(W, 0.0)
    return W


# ------------------------------------------------------------ clustering ----
def _kmeans(X: np.ndarray, k: int, rng: np.random.Generator, iters: int = 50) -> np.ndarray:
    n = X.shape[0]
    # k-means++ seeding
    centres = [X[rng.integers(n)]]
    for _ in range(1, k):
        d2 = np.min([np.sum((X - c) ** 2, axis=1) for c in centres], axis=0)
        tot = d2.sum()
        centres.append(X[rng.integers(n)] if tot <= 0 else X[rng.choice(n, p=d2 / tot)])
    C = np.array(centres)
    lab = np.zeros(n, dtype=np.int64)
    for _ in range(iters):
        new = np.argmin(((X[:, None, :] - C[None, :, :]) ** 2).sum(axis=2), axis=1)
        if np.array_equal(new, lab) and _ > 0:
            break
        lab = new
        for j in range(k):
            if np.any(lab == j):
                C[j] = X[lab == j].mean(axis=0)
    return lab


def spectral_labels(W: np.ndarray, k: int, rng: np.random.Generator) -> np.ndarray:
    """Spectral clustering with a precomputed affinity: k-means on the rows
    of the k lowest eigenvectors of the normalised Laplacian."""
    n = W.shape[0]
    if k >= n:
        return np.arange(n)
    d = W.sum(axis=1)
    dm = np.where(d > 0, 1.0 / np.sqrt(np.maximum(d, 1e-300)), 0.0)
    Lsym = np.eye(n) - dm[:, None] * W * dm[None, :]
    w, V = np.linalg.eigh(Lsym)
    X = V[:, :k]
    nrm = np.linalg.norm(X, axis=1, keepdims=True)
    X = X / np.where(nrm > 0, nrm, 1.0)
    return _kmeans(X, k, rng)


def reduce_to_two(labels: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Agglomerate cluster labels into two groups of balanced size: clusters in
    descending size go to the smaller group (on a tie, to the group they are
    more similar to)."""
    ids = list(np.unique(labels))
    ids.sort(key=lambda c: -int(np.sum(labels == c)))
    group = {}
    size = [0, 0]
    members = [np.zeros(len(labels), bool), np.zeros(len(labels), bool)]
    for c in ids:
        m = labels == c
        if size[0] != size[1]:
            g = 0 if size[0] < size[1] else 1
        else:
            aff = [W[np.ix_(m, members[j])].sum() for j in (0, 1)]
            g = 0 if aff[0] >= aff[1] else 1
        group[c] = g
        size[g] += int(m.sum())
        members[g] |= m
    return np.array([group[c] for c in labels], dtype=np.int64)


def _create_subtree(qubits, layer, W, rng):
    """Nested lists: a leaf is a qubit index, a node the list of its children."""
    if layer == 1 or len(qubits) <= 2:
        if layer == 1:
            return list(qubits)
        return [_create_subtree([q], layer - 1, W, rng) for q in qubits]
    cap = 2 ** (layer - 1)
    sub = W[np.ix_(qubits, qubits)]
    two = None
    for k in range(2, len(qubits) + 1):
        lab = reduce_to_two(spectral_labels(sub, k, rng), sub)
        if np.sum(lab == 0) <= cap and np.sum(lab == 1) <= cap:
            two = lab
            break
    if two is None:
        perm = rng.permutation(len(qubits))
        two = np.zeros(len(qubits), dtype=np.int64)
        two[perm[len(qubits) // 2:]] = 1
    q = np.asarray(qubits)
    return [_create_subtree(list(q[two == g]), layer - 1, W, rng) for g in (0, 1) if np.any(two == g)]


def _assign(node, layer, base, out):
    if not isinstance(node, list):
        out[node] = base
        return
    if layer == 0:
        raise ValueError("tree too shallow")
    half = 2 ** (layer - 1)
    for i, child in enumerate(node):
        _assign(child, layer - 1, base + i * half, out)


def clustered_layout(ops: np.ndarray, n_qubits: int, rng: np.random.Generator) -> np.ndarray:
    """One candidate layout from Algorithm 1 (random choices from rng)."""
    L = n_leaves_for(n_qubits)
    D = int(round(np.log2(L)))
    W = similarity_matrix(ops, n_qubits)
    tree = _create_subtree(list(range(n_qubits)), D, W, rng)
    out = np.full(n_qubits, -1, dtype=np.int32)
    _assign(tree, D, 0, out)
    if np.any(out < 0) or len(set(out.tolist())) != n_qubits:
        raise RuntimeError("layout construction failed")
    return out


# ---------------------------------------------------- exact bond dimension ----
def _rank(vectors) -> int:
    basis = {}
    r = 0
    for v in vectors:
        while v:
            h = v.bit_length() - 1
            if h in basis:
                v ^= basis[h]
            else:
                basis[h] = v
                r += 1
                break
    return r


def exact_bond_dim(ops: np.ndarray, n_qubits: int, leaf_of_qubit) -> int:
    """Largest Schmidt rank over every tree bond and every time of the
    circuit's Clifford skeleton (stabilizer generators as x / z bit masks;
    signs play no part in Schmidt ranks, so a reset is a measurement in the
    new basis)."""
    ops = np.asarray(ops)
    N = n_qubits
    L = n_leaves_for(N)
    leaf = np.asarray(leaf_of_qubit)
    # qubit mask below every node
    below = [0] * (2 * L)
    for q in range(N):
        below[L + int(leaf[q])] |= 1 << q
    for node in range(L - 1, 0, -1):
        below[node] = below[2 * node] | below[2 * node + 1]
    nq_below = [bin(m).count("1") for m in below]
    X = [0] * N
    Z = [1 << i for i in range(N)]

    def entropy(mask):
        k = nq_below_mask(mask)
        return _rank([(X[i] & mask) | ((Z[i] & mask) << N) for i in range(N)]) - k

    def nq_below_mask(mask):
        return bin(mask).count("1")

    def measure(q, basis):
        bit = 1 << q
        anti = [i for i in range(N) if ((X[i] if basis == 0 else Z[i]) & bit)]
        if not anti:
            return
        i0 = anti[0]
        for i in anti[1:]:
            X[i] ^= X[i0]
            Z[i] ^= Z[i0]
        X[i0], Z[i0] = (0, bit) if basis == 0 else (bit, 0)

    best = 1
    for row in ops:
        op, q0, q1 = int(row[C_OP]), int(row[C_Q0]), int(row[C_Q1])
        if op == OP_CNOT:
            cb, tb = 1 << q0, 1 << q1
            for i in range(N):
                if X[i] & cb:
                    X[i] ^= tb
                if Z[i] & tb:
                    Z[i] ^= cb
            # only bonds that separate the two qubits can change
            a, b = L + int(leaf[q0]), L + int(leaf[q1])
            path = []
            while a != b:
                if a > b:
                    path.append(a)
                    a //= 2
                else:
                    path.append(b)
                    b //= 2
            for node in path:
                if node >= L or nq_below[node] == 0 or nq_below[node] == N:
                    continue
                best = max(best, 2 ** entropy(below[node]))
        elif op == OP_MEAS:
            measure(q0, int(row[C_ARG]))
        elif op == OP_INIT:
            measure(q0, int(row[C_ARG]))
    return int(best)


def optimized_layout(ops: np.ndarray, n_qubits: int, candidates: int = 8, seed: int = 0):
    """Best of `candidates` clustered layouts by exact bond dimension.
    Returns (leaf_of_qubit, chi_exact)."""
    rng = np.random.default_rng(seed)
    best, best_chi = None, None
    for _ in range(candidates):
        lay = clustered_layout(ops, n_qubits, rng)
        chi = exact_bond_dim(ops, n_qubits, lay)
        if best_chi is None or chi < best_chi:
            best, best_chi = lay, chi
    return best, best_chi
