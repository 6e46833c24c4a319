"""Triangular hexagonal (6.6.6) colour code geometry.

The paper studies the [[(3d^2+1)/4, 1, d]] family (Sec. II.A; App. A.1,
Fig. 6): data qubits sit on the vertices of a honeycomb patch cut into a
triangle, every hexagonal face (plaquette) carries one X-type and one Z-type
check on its vertices, boundary faces have weight 4 and bulk faces weight 6.
The paper gives only the counts and a d=3 picture, so the patch is built
here from the triangular lattice: points (i, j) with i, j >= 0 and
i + j <= 3(d-1)/2.  Points with (i - j) mod 3 == 1 are face centres; every
other point is a data qubit.  A face's support is its in-patch lattice
neighbours, which are exactly the vertices of its hexagon (a honeycomb is a
triangular lattice with one of its three sublattices removed).

Qubit labels follow a row sweep over the lattice points (j outer, i inner);
a face centre contributes its X-ancilla and then its Z-ancilla at that point
of the sweep, so ancillas are labelled next to the data they touch.  This is
the "default" ordering used for the qubit-to-leaf map (qubit i on leaf i,
empty leaves on the right, App. B / Table III).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_NEIGH = ((1, 0), (-1, 0), (0, 1), (0, -1), (1, -1), (-1, 1))


@dataclass
class ColorCode:
    d: int
    n: int                      # data qubits
    n_plaq: int                 # plaquettes (faces)
    checks: np.ndarray          # [n_plaq, n] uint8 incidence (same for X and Z)
    colour: np.ndarray          # [n_plaq] face colour 0/1/2
    # global labels (0..N-1) in the default sweep order
    data_label: np.ndarray      # [n] global label of data qubit k
    xanc_label: np.ndarray      # [n_plaq] global label of the X-ancilla of face p
    zanc_label: np.ndarray      # [n_plaq] global label of the Z-ancilla of face p
    coords: dict = field(default_factory=dict)   # global label -> (i, j)

    @property
    def n_qubits(self) -> int:
        return self.n + 2 * self.n_plaq


def build_color_code(d: int) -> ColorCode:
    if d < 3 or d % 2 == 0:
        raise ValueError("distance must be odd and >= 3")
    m = 3 * (d - 1) // 2
    pts = [(i, j) for j in range(m + 1) for i in range(m + 1 - j)]
    inside = set(pts)
    is_face = {p: ((p[0] - p[1]) % 3 == 1) for p in pts}
    data_pts = [p for p in pts if not is_face[p]]
    face_pts = [p for p in pts if is_face[p]]
    data_idx = {p: k for k, p in enumerate(data_pts)}
    n, P = len(data_pts), len(face_pts)
    checks = np.zeros((P, n), dtype=np.uint8)
    colour = np.zeros(P, dtype=np.int64)
    for f, (i, j) in enumerate(face_pts):
        for di, dj in _NEIGH:
            q = (i + di, j + dj)
            if q in inside:
                checks[f, data_idx[q]] = 1
        colour[f] = (i - 1) % 3
    # default sweep labels
    data_label = np.zeros(n, dtype=np.int64)
    xanc = np.zeros(P, dtype=np.int64)
    zanc = np.zeros(P, dtype=np.int64)
    coords = {}
    lab = 0
    face_idx = {p: f for f, p in enumerate(face_pts)}
    for p in pts:
        if is_face[p]:
            f = face_idx[p]
            xanc[f] = lab
            zanc[f] = lab + 1
            coords[lab] = p
            coords[lab + 1] = p
            lab += 2
        else:
            data_label[data_idx[p]] = lab
            coords[lab] = p
            lab += 1
    return ColorCode(d=d, n=n, n_plaq=P, checks=checks, colour=colour,
                     data_label=data_label, xanc_label=xanc, zanc_label=zanc,
                     coords=coords)


def gf2_rank(mat: np.ndarray) -> int:
    """Rank over GF(2) by Gaussian elimination (rows are vectors)."""
    a = (np.array(mat, dtype=np.uint8) & 1).copy()
    rows, cols = a.shape
    r = 0
    for c in range(cols):
        piv = None
        for i in range(r, rows):
            if a[i, c]:
                piv = i
                break
        if piv is None:
            continue
        if piv != r:
            a[[r, piv]] = a[[piv, r]]
        for i in range(rows):
            if i != r and a[i, c]:
                a[i] ^= a[r]
        r += 1
        if r == rows:
            break
    return r
