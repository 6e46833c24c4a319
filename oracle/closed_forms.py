"""Values the paper's equations fix in closed form (used as pins).

SRX (Eq. 1), with U = exp(-i theta X / 2): k coherent rotations compose to
exp(-i k theta X / 2), so |0> measured in Z gives 1 with probability
sin^2(k theta / 2).  Its twirl (Eq. 9) is an X flip with p = sin^2(theta / 2);
k independent flips give 1 with probability (1 - (1 - 2p)^k) / 2.

AD (Eq. 2-3): the excited population decays as (1 - gamma)^k after k
applications and the coherence rho_01 of |+> as (1 - gamma)^(k/2) / 2.  The
jump probability of one application is gamma <n_1>: gamma on |1>, gamma / 2 on
|+>.  Twirl: p_X = p_Y = gamma / 4, p_Z = (1 - sqrt(1 - gamma))^2 / 4,
p_I = (1 + sqrt(1 - gamma))^2 / 4.

Trotterised AD (Sec. III.C, the reading with the no-jump gate
M = diag(1, e^{-gamma/2})): starting from cos(t/2)|0> - i sin(t/2)|1> (one
SRX of angle t on |0>), no jump has probability 1 - gamma sin^2(t/2) and
leaves amplitudes proportional to (cos(t/2), -i sin(t/2) e^{-gamma/2}), so a Z
measurement then reads 1 with probability
sin^2 e^{-gamma} / (cos^2 + sin^2 e^{-gamma}); the exact Kraus branch K0
gives sin^2 (1 - gamma) / (cos^2 + sin^2 (1 - gamma)) instead.

Noiseless syndrome circuit (Sec. III, App. A.1): the data start in |0...0>,
so every Z check reads +1 and Z-bar = +1; the first round's X checks are
uniformly random and later rounds repeat them; the final data bits are
uniform over the X-check row space.  Every valid record has probability
2^-P at C=1 and the same at any C (later outcomes are deterministic), so
log P = -P ln 2 for the X syndromes plus -P ln 2 for the final data bits,
i.e. -2 P ln 2, independent of C.
"""
from __future__ import annotations

import numpy as np


def srx_flip_prob(theta: float, k: int) -> float:
    return float(np.sin(k * theta / 2.0) ** 2)


def pta_srx_flip_prob(theta: float, k: int) -> float:
    p = np.sin(theta / 2.0) ** 2
    return float((1.0 - (1.0 - 2.0 * p) ** k) / 2.0)


def ad_excited_population(gamma: float, k: int) -> float:
    return float((1.0 - gamma) ** k)


def ad_plus_coherence(gamma: float, k: int) -> float:
    return float(0.5 * (1.0 - gamma) ** (k / 2.0))


def ad_jump_prob_one(gamma: float) -> float:
    return float(gamma)


def ad_jump_prob_plus(gamma: float) -> float:
    return float(gamma / 2.0)


def pta_ad_probs(gamma: float) -> np.ndarray:
    s = np.sqrt(1.0 - gamma)
    return np.array([(1 + s) ** 2 / 4, gamma / 4, gamma / 4, (1 - s) ** 2 / 4])


def noiseless_logp(n_plaq: int) -> float:
    return float(-2.0 * n_plaq * np.log(2.0))


def ad_nojump_then_one(theta: float, gamma: float, mode: str = "kraus") -> tuple:
    """(P(no jump), P(Z = 1 | no jump)) after one SRX(theta) on |0> and one AD
    location, for the exact Kraus unravelling or the Trotterised no-jump gate."""
    c2, s2 = np.cos(theta / 2.0) ** 2, np.sin(theta / 2.0) ** 2
    w = (1.0 - gamma) if mode == "kraus" else np.exp(-gamma)
    return float(1.0 - gamma * s2), float(s2 * w / (c2 + s2 * w))
