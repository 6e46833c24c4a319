"""The paper's studies on the batched engine (one GPU), as functions that
return plain dicts, and a command line that writes them as JSON.

* pta_comparison: logical failure rate of the non-Pauli channel against its
  Pauli-twirled approximation (Sec. IV.C, Eq. 9, Fig. 5) at fixed strengths,
  across code distances, one round (C = 1), clustered layout.
* truncation_background: the noiseless circuit's failure rate against the
  bond dimension chi (Sec. IV.A, Fig. 2), default layout (layout
  optimisation off), one round.
* exact_bond_dimension: the largest Schmidt rank reached by untruncated
  amplitude-damping trajectories for a qubit-to-leaf ordering (App. B,
  Table III), measured on the engine's bonds.
* threshold_sweep: failure rates over a grid of noise strengths at d = 3, 5
  and the fit of Eq. 8 (threshold tau and exponent nu, Table I).
* distance7: the d = 7 workload at chi = 128 (73 qubits, 7 rounds, SRX
  theta = 0.08 and amplitude damping gamma = 3e-3 at every location,
  clustered layout), run in the largest batches that fit the device: its
  failure rate, throughput and device memory per trajectory.
* srx_grid_vs_twirl: the d = 5, 5-round SRX workload over its theta grid
  (chi = 64, clustered layout) against the Pauli-twirled version of the same
  channel on the same random streams, per theta (the twirl as the baseline,
  Sec. IV.C, Eq. 9).

Every figure is a logical failure rate of the final-data lookup decoder with
its 99% Wilson interval; the paper's own decoder and schedule are not
available, so the values are this schedule's, not Table I's or Fig. 5's.

Usage:  python -m paper_2511_05719_amd.studies {pta,truncation,table3,threshold,d7,grid} [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from .engine import TTNEngine

Z99 = 2.5758293035489004


def wilson(k: int, n: int, z: float = Z99) -> tuple:
    """Score interval of a binomial proportion k / n (two-sided, normal
    quantile z)."""
    if n == 0:
        return 0.0, 1.0
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return max(0.0, c - h), min(1.0, c + h)


def failure_rate(circ, shots: int, theta: float, gamma: float, chi: int, dtype: str = "c64",
                 cutoff: float = 1e-10, batch: int = 2048, seed: int = 0, traj_offset: int = 0) -> dict:
    """Run `shots` trajectories of the circuit in batches and decode them."""
    batch = min(batch, shots)
    eng = TTNEngine(circ.n_qubits, batch, circ.leaf_of_qubit, chi_max=chi, cutoff=cutoff, dtype=dtype, seed=seed)
    ol = eng.upload(circ)
    fails = done = 0
    disc = 0.0
    max_rank = 1
    t0 = time.perf_counter()
    while done < shots:
        res = eng.run_circuit(ol, theta=theta, gamma=gamma, traj_offset=traj_offset + done, stats=True)
        f = eng.decode(res.records, circ.data_rec, circ.code.checks).cpu().numpy()
        take = min(batch, shots - done)
        fails += int(f[:take].sum())
        done += take
        disc += res.stats["discarded_weight"] * take / batch
        max_rank = max(max_rank, res.stats["max_rank"])
        print(f"  {done}/{shots} shots, {fails} failures, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    eng.close()
    lo, hi = wilson(fails, done)
    return {"shots": done, "failures": fails, "p_fail": fails / done, "ci99": [lo, hi],
            "mean_discarded_weight": disc / done, "max_rank": max_rank, "seconds": dt}


def pta_comparison(distances=(3, 5), shots: int = 10000, theta: float = 2 * math.pi * 1e-2, gamma: float = 4e-3,
                   chi: int = 64, rounds: int = 1, seed: int = 5) -> dict:
    """Fig. 5 settings: SRX with theta_paper / pi = 1e-2 (theta = 2 pi 1e-2 rad
    in the exp(-i theta X / 2) convention), AD with gamma = 4e-3, C = 1; each
    channel against its Pauli twirl on the same random streams."""
    from workload import build_circuit
    out = {"settings": {"theta_rad": theta, "theta_paper_over_pi": theta / 2 / math.pi, "gamma": gamma,
                        "rounds": rounds, "chi_max": chi, "cutoff": 1e-10, "dtype": "c64",
                        "layout": "clustered (App. B, Algorithm 1)", "shots_per_point": shots,
                        "decoder": "final-data lookup (minimum-weight leader)", "seed": seed},
           "points": []}
    for d in distances:
        for model, exact, twirl, th, ga in (("SRX", "srx", "pta_srx", theta, 0.0), ("AD", "ad", "pta_ad", 0.0, gamma)):
            row = {"d": d, "model": model}
            for tag, ch in (("exact", exact), ("pta", twirl)):
                circ = build_circuit(d, rounds, ch, leaf_of_qubit="optimized")
                row[tag] = failure_rate(circ, shots, th, ga, chi, seed=seed)
            out["points"].append(row)
            print(json.dumps(row), flush=True)
    return out


def srx_grid_vs_twirl(thetas=tuple(0.02 + i * 0.18 / 7 for i in range(8)), shots: int = 10000, d: int = 5,
                      rounds: int = 5, chi: int = 64, batch: int = 4096, seed: int = 2) -> dict:
    """The SRX channel at every theta of the grid against its Pauli twirl
    (Eq. 9: X flips with p = sin^2(theta / 2)), each on `shots` trajectories
    of the same random streams, clustered layout, complex64, cutoff 1e-10.
    The twirled circuit stays a stabilizer state, so chi never binds there;
    the coherent one is truncated at chi."""
    from workload import build_circuit
    out = {"settings": {"d": d, "rounds": rounds, "chi_max": chi, "cutoff": 1e-10, "dtype": "c64",
                        "layout": "clustered (App. B, Algorithm 1)", "shots_per_point": shots, "seed": seed,
                        "decoder": "final-data lookup (minimum-weight leader)"},
           "points": []}
    circs = {ch: build_circuit(d, rounds, ch, leaf_of_qubit="optimized") for ch in ("srx", "pta_srx")}
    for j, th in enumerate(thetas):
        row = {"theta": float(th)}
        for tag, ch in (("srx", "srx"), ("twirl", "pta_srx")):
            row[tag] = failure_rate(circs[ch], shots, float(th), 0.0, chi, seed=seed, batch=batch,
                                    traj_offset=j << 32)
        out["points"].append(row)
        print(json.dumps({"theta": row["theta"], "srx": row["srx"]["p_fail"], "twirl": row["twirl"]["p_fail"]}),
              flush=True)
    return out


def truncation_background(d: int, chis, shots: int, rounds: int = 1, seed: int = 6, batch: int = 2048) -> dict:
    """Fig. 2: the noiseless circuit, default layout (optimisation off); the
    exact bond dimension is that of the Clifford circuit (stabilizer ranks)."""
    from workload import build_circuit, exact_bond_dim
    circ = build_circuit(d, rounds, "none")
    chi_exact = exact_bond_dim(circ.ops, circ.n_qubits, circ.leaf_of_qubit)
    out = {"d": d, "rounds": rounds, "layout": "default (qubit i on leaf i)", "chi_exact": chi_exact,
           "dtype": "c64", "cutoff": 1e-10, "seed": seed, "points": []}
    for chi in chis:
        b = batch if chi <= 64 else min(batch, 512)
        r = failure_rate(circ, shots, 0.0, 0.0, chi, seed=seed, batch=b)
        r.update({"chi": chi, "chi_over_chi_exact": chi / chi_exact})
        out["points"].append(r)
        print(json.dumps({"d": d, "chi": chi, "p_fail": r["p_fail"], "ci99": r["ci99"]}), flush=True)
    return out


def exact_bond_dimension(d: int, rounds: int, layout: str, chi: int, gamma: float = 1e-2, rows: int = 32,
                         cutoff: float = 1e-14, seed: int = 7) -> dict:
    """Largest Schmidt rank over every bond and time of `rows` AD trajectories
    run with the cap chi and a cutoff that drops only numerical zeros; a
    result equal to chi means the cap was reached (chi_exact >= chi)."""
    from workload import build_circuit
    circ = build_circuit(d, rounds, "ad", leaf_of_qubit=layout)
    eng = TTNEngine(circ.n_qubits, rows, circ.leaf_of_qubit, chi_max=chi, cutoff=cutoff, dtype="c128", seed=seed)
    res = eng.run_circuit(eng.upload(circ), theta=0.0, gamma=gamma, stats=True)
    torch.cuda.synchronize()
    st = res.stats
    eng.close()
    return {"d": d, "rounds": rounds, "layout": layout, "gamma": gamma, "rows": rows, "chi_cap": chi,
            "max_rank": st["max_rank"], "cap_reached": st["max_rank"] >= chi,
            "discarded_weight_per_row": st["discarded_weight"] / rows}


def threshold_ansatz(X, A, B, C, tau, nu):
    """Eq. 8: p_fail = A + B x + C x^2 with x = (p_err - tau) d^(1/nu)."""
    p, d = X
    x = (p - tau) * d ** (1.0 / nu)
    return A + B * x + C * x * x


def fit_threshold(points, tau0: float) -> dict:
    """Weighted least-squares fit of Eq. 8 to (d, p_err, failures, shots)
    points; the 99% interval of tau is the normal one from the fit's
    covariance (binomial variances of the points, floored at one event)."""
    from scipy.optimize import curve_fit
    p = np.array([q["p_err"] for q in points], dtype=float)
    d = np.array([q["d"] for q in points], dtype=float)
    k = np.array([q["failures"] for q in points], dtype=float)
    n = np.array([q["shots"] for q in points], dtype=float)
    y = k / n
    sig = np.sqrt(np.maximum(y * (1 - y), 1.0 / n) / n)
    popt, pcov = curve_fit(threshold_ansatz, (p, d), y, p0=[float(np.mean(y)), 1.0, 0.0, tau0, 1.0],
                           sigma=sig, absolute_sigma=True, maxfev=20000)
    err = np.sqrt(np.maximum(np.diag(pcov), 0.0))
    chi2 = float(np.sum(((threshold_ansatz((p, d), *popt) - y) / sig) ** 2))
    names = ("A", "B", "C", "tau", "nu")
    return {"params": dict(zip(names, map(float, popt))), "stderr": dict(zip(names, map(float, err))),
            "tau_ci99": [float(popt[3] - Z99 * err[3]), float(popt[3] + Z99 * err[3])],
            "chi2": chi2, "dof": int(len(y) - len(popt))}


def crossing(points) -> float:
    """Noise strength where the failure-rate curves of the smallest and the
    largest distance cross (linear interpolation between the two grid points
    around the first sign change of their difference), or nan."""
    ds = sorted({q["d"] for q in points})
    lo, hi = ds[0], ds[-1]
    a = {q["p_err"]: q["p_fail"] for q in points if q["d"] == lo}
    b = {q["p_err"]: q["p_fail"] for q in points if q["d"] == hi}
    ps = sorted(set(a) & set(b))
    diff = [b[p] - a[p] for p in ps]
    for i in range(len(ps) - 1):
        if diff[i] < 0 <= diff[i + 1]:
            return float(ps[i] + (ps[i + 1] - ps[i]) * (-diff[i]) / (diff[i + 1] - diff[i]))
    return float("nan")


def _sweep(model, strengths, distances, rounds, shots, chi, seed, tag):
    from workload import build_circuit
    ch = {"SRX": "srx", "AD": "ad"}[model]
    pts = []
    for d in distances:
        circ = build_circuit(d, rounds, ch, leaf_of_qubit="optimized")
        for j, v in enumerate(strengths):
            th, ga = (v, 0.0) if model == "SRX" else (0.0, v)
            r = failure_rate(circ, shots, th, ga, chi, seed=seed, traj_offset=(tag << 40) | (j << 32))
            r.update({"d": d, "p_err": float(v)})
            pts.append(r)
            print(json.dumps({"model": model, "d": d, "p_err": v, "p_fail": r["p_fail"], "ci99": r["ci99"]}),
                  flush=True)
    return pts


def threshold_sweep(model: str, strengths, distances=(3, 5), rounds: int = 1, shots: int = 10000, chi: int = 64,
                    seed: int = 8, fine_points: int = 8) -> dict:
    """Failure rates over a coarse grid of noise strengths at several
    distances (Sec. IV.B, Fig. 3), the crossing of the smallest and largest
    distance, a fine grid over [0.5, 1.5] x the crossing, and the fit of
    Eq. 8 (threshold tau and exponent nu, Table I) to the fine grid, where the
    quadratic ansatz applies; model "SRX" (theta in rad, exp(-i theta X / 2))
    or "AD" (gamma)."""
    coarse = _sweep(model, strengths, distances, rounds, shots, chi, seed, 1)
    tau0 = crossing(coarse)
    out = {"model": model, "rounds": rounds, "chi_max": chi, "layout": "clustered (App. B, Algorithm 1)",
           "decoder": "final-data lookup (minimum-weight leader)", "shots_per_point": shots,
           "coarse": coarse, "crossing": tau0}
    if not math.isfinite(tau0):
        out["fit_eq8"] = {"error": "the curves do not cross on the coarse grid"}
        return out
    fine = _sweep(model, np.linspace(0.5 * tau0, 1.5 * tau0, fine_points), distances, rounds, shots, chi, seed, 2)
    out["fine"] = fine
    try:
        out["fit_eq8"] = fit_threshold(fine, tau0)
    except Exception as e:            # the fit did not converge: report it
        out["fit_eq8"] = {"error": str(e)}
    return out


def distance7(shots: int = 4096, rounds: int = 7, theta: float = 0.08, gamma: float = 3e-3, chi: int = 128,
              batch: int = 256, seed: int = 3) -> dict:
    """The d = 7 colour code at chi = 128 in batches of `batch` rows: a node
    buffer holds its largest shape (two legs at 2 chi on a controlled gate's
    path) for every row, ~643 MiB per row here, so a context takes a few
    hundred rows and the shots run as consecutive batches (trajectory ids
    continue across batches, so the result does not depend on the split)."""
    from workload import build_circuit
    circ = build_circuit(7, rounds, "srx+ad", leaf_of_qubit="optimized")
    batch = min(batch, shots)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    eng = TTNEngine(circ.n_qubits, batch, circ.leaf_of_qubit, chi_max=chi, cutoff=1e-10, dtype="c64", seed=seed)
    free1, _ = torch.cuda.mem_get_info()
    ol = eng.upload(circ)
    fails = done = 0
    disc = 0.0
    max_rank = 1
    t0 = time.perf_counter()
    while done < shots:
        res = eng.run_circuit(ol, theta=theta, gamma=gamma, traj_offset=done, stats=True)
        f = eng.decode(res.records, circ.data_rec, circ.code.checks).cpu().numpy()
        take = min(batch, shots - done)
        fails += int(f[:take].sum())
        done += take
        disc += res.stats["discarded_weight"] * take / batch
        max_rank = max(max_rank, res.stats["max_rank"])
        print(f"  {done}/{shots} shots, {fails} failures, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    eng.close()
    lo, hi = wilson(fails, done)
    n_ops = len(circ.ops)
    return {"study": "d = 7 colour code at chi = 128 (config 4 shape)", "d": 7, "qubits": circ.n_qubits,
            "rounds": rounds, "theta": theta, "gamma": gamma, "chi_max": chi, "layout": "clustered",
            "dtype": "c64", "batch": batch, "shots": done, "failures": fails, "p_fail": fails / done,
            "ci99": [lo, hi], "mean_discarded_weight": disc / done, "max_rank": max_rank, "seconds": dt,
            "shots_per_s": done / dt, "trajectory_gates_per_s": done * n_ops / dt, "ops_per_shot": n_ops,
            "device_gib": (free0 - free1) / 2 ** 30, "device_mib_per_row": (free0 - free1) / 2 ** 20 / batch}


def main(argv=None):
    ap = argparse.ArgumentParser(description="the paper's studies on the batched engine")
    ap.add_argument("study", choices=("pta", "truncation", "table3", "threshold", "d7", "grid"))
    ap.add_argument("--out", default=None)
    ap.add_argument("--shots", type=int, default=None)
    ap.add_argument("--batch", type=int, default=None)
    a = ap.parse_args(argv)
    if a.study == "d7":
        res = distance7(shots=a.shots or 4096, batch=a.batch or 256)
    elif a.study == "grid":
        res = srx_grid_vs_twirl(shots=a.shots or 10000, batch=a.batch or 4096)
    elif a.study == "pta":
        res = pta_comparison(shots=a.shots or 10000)
    elif a.study == "truncation":
        res = {"studies": [truncation_background(3, (1, 2, 4, 8), a.shots or 10000),
                           truncation_background(5, (1, 2, 4, 8, 16, 32, 64, 128), a.shots or 4096)]}
    elif a.study == "threshold":
        res = {"sweeps": [threshold_sweep("SRX", np.linspace(0.005, 0.08, 8), shots=a.shots or 10000),
                          threshold_sweep("AD", np.geomspace(1e-3, 4e-2, 8), shots=a.shots or 10000)]}
    else:
        pts = []
        for d, C, chi in ((3, 1, 64), (3, 3, 64), (5, 1, 128)):
            for lay in ("default", "snake", "optimized"):
                p = exact_bond_dimension(d, C, lay, chi)
                pts.append(p)
                print(json.dumps(p), flush=True)
        res = {"study": "exact bond dimension of amplitude-damping trajectories (Table III)", "points": pts}
    res["device"] = torch.cuda.get_device_name(0)
    text = json.dumps(res, indent=1)
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as f:
            f.write(text + "\n")
    else:
        print(text)


if __name__ == "__main__":
    sys.exit(main())
