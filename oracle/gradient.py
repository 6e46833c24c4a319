"""Derivatives of log P(record) by the per-location noise parameters.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a given record -- the measurement bits and, under amplitude damping, the
Kraus branch of every AD op -- the probability is P = <psi_N|psi_N>, psi_N the
unnormalised state after all ops with the recorded outcomes forced
(statevector.run with forced records returns log P as the sum of the log
conditional probabilities).  One location's parameter enters P through a
single 2 x 2 operator, applied on the ket and on the bra, which fixes how P
depends on it:

* SRX at location l (Eq. 1): U(t) = cos(t/2) I - i sin(t/2) X, so
  P(t) = a + b cos t + c sin t and dP/dt = (P(t + pi/2) - P(t - pi/2)) / 2
  holds exactly.
* Amplitude damping (Eq. 2-3), recorded branch "no jump":
  K0 = |0><0| + s |1><1| with s = sqrt(1 - gamma), so P = a + b s + c s^2.
  A quadratic is fixed by three values; the one-sided three-point rule
  dP/ds = (3 P(s) - 4 P(s - h) + P(s - 2h)) / (2h) is exact for it, and
  dP/dgamma = -dP/ds / (2 s).
* Recorded branch "jump": K1 = sqrt(gamma) |0><1|, so P is proportional to
  gamma and d log P / d gamma = 1 / gamma.

d log P = dP / P.  Every shifted parameter set is one row of a single batched
statevector run with the same forced record.  (Each location must carry at
most one SRX op and one AD op, as in the colour-code circuits.)
"""
from __future__ import annotations

import numpy as np

from . import statevector as sv

OP_SRX, OP_AD = 2, 3
C_OP, C_LOC = 0, 4


def log_prob_grad(circ, theta, gamma, record, branch=None):
    """One trajectory: theta, gamma [n_loc]; record [n_rec]; branch [n_ad].

    Returns (log P, dlogP/dtheta [n_loc], dlogP/dgamma [n_loc])."""
    ops = np.asarray(circ.ops)
    th0 = np.asarray(theta, dtype=np.float64).reshape(-1)
    ga0 = np.asarray(gamma, dtype=np.float64).reshape(-1)
    n_loc = circ.n_loc
    rec = np.asarray(record, dtype=np.uint8).reshape(1, -1)
    br = None if circ.n_ad == 0 else np.asarray(branch, dtype=np.int8).reshape(1, -1)

    srx_locs = [int(l) for l in ops[ops[:, C_OP] == OP_SRX, C_LOC]]
    ad_rows = np.nonzero(ops[:, C_OP] == OP_AD)[0]
    ad_locs = [int(ops[k, C_LOC]) for k in ad_rows]
    if len(set(srx_locs)) != len(srx_locs) or len(set(ad_locs)) != len(ad_locs):
        raise ValueError("a location carries more than one op of a channel")
    ad_jump = {} if br is None else {loc: bool(br[0, j]) for j, loc in enumerate(ad_locs)}

    # rows: 0 = base, then 2 per SRX location, 2 per no-jump AD location
    thetas, gammas, tags = [th0.copy()], [ga0.copy()], [("base", -1, 0.0)]
    for l in srx_locs:
        for sgn in (+1, -1):
            t = th0.copy()
            t[l] += sgn * np.pi / 2
            thetas.append(t)
            gammas.append(ga0.copy())
            tags.append(("srx", l, sgn))
    for l in ad_locs:
        if ad_jump.get(l, False):
            continue
        s0 = np.sqrt(1.0 - ga0[l])
        h = s0 / 4.0
        for m in (1, 2):
            g = ga0.copy()
            g[l] = 1.0 - (s0 - m * h) ** 2
            thetas.append(th0.copy())
            gammas.append(g)
            tags.append(("ad", l, m))
    T = len(tags)
    res = sv.run(circ, np.stack(thetas), np.stack(gammas), 0, np.arange(T),
                 forced_records=np.repeat(rec, T, axis=0),
                 forced_branches=None if br is None else np.repeat(br, T, axis=0))
    logp = res.logp
    P0 = np.exp(logp[0])
    dth = np.zeros(n_loc)
    dga = np.zeros(n_loc)
    plus, minus, ad1, ad2 = {}, {}, {}, {}
    for i, (kind, l, m) in enumerate(tags):
        if kind == "srx":
            (plus if m > 0 else minus)[l] = np.exp(logp[i])
        elif kind == "ad":
            (ad1 if m == 1 else ad2)[l] = np.exp(logp[i])
    for l in srx_locs:
        dth[l] = 0.5 * (plus[l] - minus[l]) / P0
    for l in ad_locs:
        if ad_jump.get(l, False):
            dga[l] = 1.0 / ga0[l]
            continue
        s0 = np.sqrt(1.0 - ga0[l])
        h = s0 / 4.0
        dPds = (3.0 * P0 - 4.0 * ad1[l] + ad2[l]) / (2.0 * h)
        dga[l] = -dPds / (2.0 * s0) / P0
    return logp[0], dth, dga


def log_prob(circ, theta, gamma, records, branches=None):
    """log P of several records [T, n_rec] (parameters [n_loc] or [T, n_loc])."""
    records = np.asarray(records, dtype=np.uint8)
    T = records.shape[0]
    res = sv.run(circ, theta, gamma, 0, np.arange(T), forced_records=records, forced_branches=branches)
    return res.logp
