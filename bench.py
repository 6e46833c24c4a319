#!/usr/bin/env python3
"""Throughput of the TTN trajectory engine on one MI355X.

Workload: the d=5 triangular colour code (37 qubits: 19 data + 18 ancillas),
5 rounds of X-then-Z syndrome extraction, a systematic X over-rotation
exp(-i theta X / 2) after every gate, initialisation and idle location with
theta cycling over an 8-point grid in [0.02, 0.2] rad across trajectories,
binary tree over 64 leaves with the clustered qubit-to-leaf layout of App. B
(Algorithm 1, the layout the paper runs its simulations on), chi_max = 64,
squared-weight cutoff 1e-10; contractions in complex64 on FP32 MFMA, Gram
matrices / eigen-decompositions / probabilities in FP64.

A step is one batched run of the whole circuit (2427 ops per trajectory:
CNOTs, noise ops, initialisations, measurements) for `--batch` trajectories.
The metric is trajectory-gates/s = trajectories/s x ops per trajectory; the
same circuit in complex128, one trajectory at a time (the plain path), and
the FP64 CPU oracle on a bounded sample are reported beside it.  Extra legs
(each run only while the wall-clock budget allows): the same workload with
the default qubit order, and log P with its adjoint gradient for records of
the differentiation workload.

Prints one JSON line.  --gpus N > 1 is not supported (one GPU per box).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "trajectory-gates/s and shots/s at d=5 chi=64, batched cplx64 vs plain cplx128"
PEAK = {"fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "fp64_valu": 78.6e12, "hbm": 8.0e12}
THETAS = [0.02 + i * (0.2 - 0.02) / 7 for i in range(8)]
# the whole command (warm-up, timed steps, statistics step and legs) is
# planned to end this many seconds after start
DEFAULT_BUDGET_S = 480.0


def elapsed() -> float:
    return time.perf_counter() - T_START


def log(*a):
    print(f"[{elapsed():7.1f}s]", *a, file=sys.stderr, flush=True)


def theta_rows(circ, rows, offset):
    import numpy as np
    th = np.asarray(THETAS)[(offset + np.arange(rows)) % len(THETAS)]
    return np.repeat(th[:, None], circ.n_loc, axis=1)


def wilson(k, n, z=2.5758293035489004):
    """99% Wilson score interval of k successes in n trials."""
    if n == 0:
        return 0.0, 1.0
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * ((p * (1 - p) / n + z * z / (4 * n * n)) ** 0.5) / den
    return max(0.0, c - h), min(1.0, c + h)


def run_batched(args, circ, budget_end):
    """Warm-up steps (the first measures GEMM tile shapes), then up to
    args.steps timed steps; a step that would end after budget_end is not
    started (the line then reports the steps actually timed)."""
    import numpy as np
    import torch
    from paper_2511_05719_amd import TTNEngine
    B = args.batch
    free0, _ = torch.cuda.mem_get_info()
    eng = TTNEngine(circ.n_qubits, B, circ.leaf_of_qubit, chi_max=64, cutoff=1e-10, dtype="c64",
                    seed=args.seed)
    free1, _ = torch.cuda.mem_get_info()
    ol = eng.upload(circ)
    params_dev = [torch.as_tensor(theta_rows(circ, B, k * B), device="cuda")
                  for k in range(args.warmup + args.steps)]
    eng.autotune(not args.no_autotune and args.warmup > 0)
    warm_s = []
    for w in range(args.warmup):
        t0 = time.perf_counter()
        eng.run_circuit(ol, theta=params_dev[w], traj_offset=w * B, stats=False)
        torch.cuda.synchronize()
        warm_s.append(time.perf_counter() - t0)
        if w == 0:
            tuned = eng.autotune(False)
        log(f"warmup step {w}: {warm_s[-1]:.2f} s")
    if args.warmup == 0:
        tuned = eng.autotune(False)
    eng.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(args.steps):
        if k > 0:
            per = (time.perf_counter() - t0) / k
            if elapsed() + per > budget_end:
                log(f"budget: stopping after {k} timed steps")
                break
        i = args.warmup + k
        results.append(eng.run_circuit(ol, theta=params_dev[i], traj_offset=i * B, stats=False))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = eng.profile_read()
    eng.profile(False)
    steps = len(results)
    log(f"timed {steps} steps in {t1 - t0:.3f} s")
    # logical failures per theta over every timed trajectory (decoded after
    # the timed region)
    fails = np.zeros(len(THETAS), dtype=np.int64)
    shots = np.zeros(len(THETAS), dtype=np.int64)
    for k, res in enumerate(results):
        f = eng.decode(res.records, circ.data_rec, circ.code.checks).cpu().numpy().astype(np.int64)
        j = (np.arange(B) + (args.warmup + k) * B) % len(THETAS)
        fails += np.bincount(j, weights=f, minlength=len(THETAS)).astype(np.int64)
        shots += np.bincount(j, minlength=len(THETAS))
    st = {}
    if elapsed() + (t1 - t0) / max(steps, 1) < budget_end + 60:
        # one more step with statistics (untimed): ranks and discarded weight
        st = eng.run_circuit(ol, theta=params_dev[args.warmup], traj_offset=args.warmup * B, stats=True).stats
    eng.close()
    st["engine_device_gib"] = (free0 - free1) / 2 ** 30
    st["autotune"] = {"shapes_measured": tuned[0], "differs_from_fixed_rule": tuned[1]}
    pf = []
    for j, th in enumerate(THETAS):
        lo, hi = wilson(int(fails[j]), int(shots[j]))
        pf.append({"theta": round(th, 5), "shots": int(shots[j]), "p_fail": fails[j] / max(shots[j], 1),
                   "ci99": [lo, hi]})
    return t1 - t0, steps, prof, st, pf, warm_s


def run_plain(args, circ):
    """The plain path: complex128, one trajectory per launch sequence, the
    same algorithm and truncation rule; shots spread over the theta grid."""
    import torch
    from paper_2511_05719_amd import TTNEngine
    eng = TTNEngine(circ.n_qubits, 1, circ.leaf_of_qubit, chi_max=64, cutoff=1e-10, dtype="c128",
                    seed=args.seed)
    ol = eng.upload(circ)
    eng.run_circuit(ol, theta=theta_rows(circ, 1, 0), traj_offset=10 ** 9, stats=False)   # warm
    torch.cuda.synchronize()
    per_theta = {}
    t0 = time.perf_counter()
    for i in range(args.plain_shots):
        ts = time.perf_counter()
        eng.run_circuit(ol, theta=theta_rows(circ, 1, i), traj_offset=i, stats=False)
        torch.cuda.synchronize()
        per_theta.setdefault(round(THETAS[i % len(THETAS)], 5), []).append(time.perf_counter() - ts)
    t1 = time.perf_counter()
    eng.close()
    return (t1 - t0) / args.plain_shots, {k: sum(v) / len(v) for k, v in per_theta.items()}


def run_layout_leg(args, layout, batch):
    """The same workload with another qubit-to-leaf layout: one warm-up step
    (tile shapes measured) and one timed step."""
    import torch
    from paper_2511_05719_amd import TTNEngine
    from workload import build_circuit, exact_bond_dim
    circ = build_circuit(5, args.rounds, "srx", leaf_of_qubit=layout)
    eng = TTNEngine(circ.n_qubits, batch, circ.leaf_of_qubit, chi_max=64, cutoff=1e-10, dtype="c64",
                    seed=args.seed)
    ol = eng.upload(circ)
    eng.autotune(not args.no_autotune)
    eng.run_circuit(ol, theta=theta_rows(circ, batch, 0), traj_offset=0, stats=False)
    torch.cuda.synchronize()
    eng.autotune(False)
    t0 = time.perf_counter()
    res = eng.run_circuit(ol, theta=theta_rows(circ, batch, batch), traj_offset=batch, stats=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = res.stats
    p_fail = float(eng.decode(res.records, circ.data_rec, circ.code.checks).float().mean().item())
    eng.close()
    shots = batch / dt
    skel = build_circuit(5, args.rounds, "none", leaf_of_qubit=circ.leaf_of_qubit)
    return {"layout": layout, "batch": batch, "steps": 1,
            "shots_per_s": shots, "trajectory_gates_per_s": shots * circ.n_ops,
            "chi_exact_clifford_skeleton": exact_bond_dim(skel.ops, circ.n_qubits, circ.leaf_of_qubit),
            "p_fail": p_fail, "mean_discarded_weight": st.get("discarded_weight", 0.0) / batch,
            "max_rank": st.get("max_rank"), "note": "the timed step includes filling the statistics"}


def run_graph_leg(args, circ, batch):
    """The same workload in the two other run modes of the batch driver: static
    shapes (no host read per centre move) eagerly, and the whole op list
    captured once into a HIP graph and replayed; one untimed call each
    (the graph mode's captures), then one timed call, against the dynamic mode."""
    import torch
    from paper_2511_05719_amd import TTNEngine
    th = torch.as_tensor(theta_rows(circ, batch, 0), device="cuda")
    eng = TTNEngine(circ.n_qubits, batch, circ.leaf_of_qubit, chi_max=64, cutoff=1e-10, dtype="c64",
                    seed=args.seed)
    ol = eng.upload(circ)
    out = eng.outputs(ol)
    res = {"batch": batch}
    for mode in ("dynamic", "static", "graph"):
        eng.run_mode(mode)
        eng.run_circuit(ol, theta=th, traj_offset=0, out=out, stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eng.run_circuit(ol, theta=th, traj_offset=batch, out=out, stats=False)
        torch.cuda.synchronize()
        res[mode + "_shots_per_s"] = batch / (time.perf_counter() - t0)
    res["graph_captures"], res["graph_replays"] = eng.run_mode("graph")
    eng.close()
    return res


def run_gradient(args):
    """log P and its adjoint gradient for records of the differentiation
    workload (d=5, 3 rounds, SRX theta = 0.1 and AD gamma = 5e-3 at every
    location, records sampled from the forward model), clustered layout."""
    import torch
    from paper_2511_05719_amd import TTNEngine
    from workload import build_circuit
    circ = build_circuit(5, 3, "srx+ad", leaf_of_qubit="optimized")
    B = args.grad_records
    eng = TTNEngine(circ.n_qubits, B, circ.leaf_of_qubit, chi_max=64, cutoff=1e-10, dtype="c64", seed=4)
    ol = eng.upload(circ)
    res = eng.run_circuit(ol, theta=0.1, gamma=5e-3, stats=False)
    rec, br = res.records.clone(), res.branches.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lp, dth, dga, st = eng.log_prob_grad(ol, rec, br, theta=0.1, gamma=5e-3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    eng.close()
    return {"workload": "d=5 colour code, 3 rounds, SRX theta=0.1 + AD gamma=5e-3, chi_max=64, complex64, "
                        "clustered layout", "records": B, "parameters_per_record": 2 * circ.n_loc,
            "seconds": dt, "records_per_s": B / dt, "flagged_rows": st.get("flagged_rows")}


def host_cpu():
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, timeout=10).stdout
        for line in out.decode(errors="replace").splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except Exception:
        nproc = os.cpu_count()
    return model, nproc


def first_full_register_op(circ) -> int:
    """Index of the first op after every data qubit and every ancilla of a
    phase are live (the oracle's register has its full n + P qubits)."""
    live = set(int(q) for q in circ.code.data_label)
    full = len(live) + circ.code.n_plaq
    for k, o in enumerate(circ.ops):
        if o[0] == 0:
            live.add(int(o[1]))
        elif o[0] == 5:
            live.discard(int(o[1]))
        if len(live) == full and o[0] != 0:
            return k
    return 0


def cpu_oracle(circ, seed, n_ops=10):
    """The FP64 oracle (lazy-ancilla state vector, numpy, one thread) on the
    same circuit: n_ops consecutive ops of one trajectory on the full 28-qubit
    live register, timed as the difference of two runs from the start."""
    import numpy as np
    from oracle import statevector as sv
    from threadpoolctl import threadpool_limits
    k0 = first_full_register_op(circ)
    ka, kb = k0 - 1, k0 - 1 + n_ops
    with threadpool_limits(1):
        t0 = time.perf_counter()
        sv.run(circ, 0.1, 0.0, seed, np.arange(1), stop_after_op=ka)
        t1 = time.perf_counter()
        sv.run(circ, 0.1, 0.0, seed, np.arange(1), stop_after_op=kb)
        t2 = time.perf_counter()
    rate = (kb - ka) / max((t2 - t1) - (t1 - t0), 1e-9)
    return rate, (t2 - t0), (ka + 1, kb)


# HBM traffic of one launch of a kernel class at this workload and batch
# (rocprofv3 FETCH_SIZE / WRITE_SIZE passes, each scaled by what the counter
# reads for a 256 MiB device copy, see the profile named), valid for the
# source file it was measured on: reported only while that file is unchanged
TRAFFIC = {
    "profile": "profiles/ttn_d5_chi64_b4096_clustered_hbm_traffic.txt",
    "batch": 4096,
    "layout": "optimized",
    "classes": {
        # k_zgemm<float2, float2, float2, float, ...>, all tile shapes: 455.7 MB read + 354.1 MB written
        "contract": {"bytes_per_launch": 809.8e6, "source": "ttn_gemm.hip",
                     "sha256": "7947118a61490b5cc3877f46a50dbbcdcd637d5e8c5e1061255deaa89beec0b3"},
        # k_zgemm<float2, float2, double2, double, ...>, all tile shapes: 382.1 MB read + 47.9 MB written
        "gram": {"bytes_per_launch": 430.0e6, "source": "ttn_gemm.hip",
                 "sha256": "7947118a61490b5cc3877f46a50dbbcdcd637d5e8c5e1061255deaa89beec0b3"},
    },
}


def class_traffic(cls, batch, layout):
    import hashlib
    ent = TRAFFIC["classes"].get(cls)
    if ent is None or batch != TRAFFIC["batch"] or layout != TRAFFIC["layout"]:
        return None
    src = os.path.join(ROOT, "paper_2511_05719_amd", "csrc", ent["source"])
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    return ent["bytes_per_launch"] if h == ent["sha256"] else None


def copy_calibration():
    """Three device copies of 256 MiB: the reference dispatch that scales the
    FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x 256 MiB", flush=True)


# machine balance: below this many algorithmic flops per algorithmic byte a
# class is bound by HBM bandwidth, above it by its MFMA pipe
RIDGE = {"contract": PEAK["fp32_mfma"] / PEAK["hbm"], "gram": PEAK["fp64_mfma"] / PEAK["hbm"]}
PER_UNIT_BYTES = {
    "contract": "8 ((n + k) r + 2 k n) bytes per centre move and side (complex64: node read once, factor read "
                "once, result written once at the actual dimensions; per diagonal block in block moves)",
    "gram": "8 n r + 16 n^2 bytes per Gram matrix (node rows read once, FP64 complex result written once)",
}
PER_UNIT = {
    "eigh": "36 n^3 real flops per n x n complex Hermitian eigen-decomposition with vectors, "
            "n = actual bond dimension (non-zero Gram eigenvalues)",
    "gram": "8 n^2 r real flops per Gram matrix (n = actual bond dimension, r = product of the other "
            "two actual leg dimensions; per diagonal block in block-diagonal moves)",
    "contract": "8 k n r real flops per factor product (k kept, n actual bond dimension, r = product "
                "of the other two actual leg dimensions)",
    "move": "8 (r^2 (3n - 2r) / 3 + r^3 / 3) real flops per exact centre move (pivoted Cholesky of "
            "rank r and the inverse of its triangle, n = problem size)",
}
BOUND_OF = {"contract": ("mfma", PEAK["fp32_mfma"]), "gram": ("mfma", PEAK["fp64_mfma"]),
            "eigh_small": ("alu", PEAK["fp64_valu"]), "eigh_large": ("alu", PEAK["fp64_valu"]),
            "move": ("alu", PEAK["fp64_valu"])}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--rounds", type=int, default=5)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--layout", choices=("optimized", "default"), default="optimized",
                    help="qubit-to-leaf layout of the headline run (App. B clustered, or qubit i on leaf i)")
    ap.add_argument("--budget", type=float, default=DEFAULT_BUDGET_S,
                    help="seconds after start by which the whole command should end")
    ap.add_argument("--plain-shots", type=int, default=16)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other-layout and gradient legs")
    ap.add_argument("--no-autotune", action="store_true", help="fixed-rule GEMM tile shapes (no measuring "
                    "in the warm-up)")
    ap.add_argument("--grad-records", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true", help="only run the 256 MiB copy that "
                    "calibrates the HBM byte counters, then exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the trajectories would "
              "shard across GPUs as contiguous id ranges, one process per GPU, with only the failure "
              "tallies all-reduced)", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs as a single process on one GPU", file=sys.stderr)
        sys.exit(2)
    from workload import build_circuit, ops_per_shot
    lay = "optimized" if args.layout == "optimized" else None
    circ = build_circuit(5, args.rounds, "srx", leaf_of_qubit=lay)
    ops = ops_per_shot(circ)
    # the batched run gets the budget minus what the legs after it need
    legs_s = (0 if args.no_plain else 25) + (0 if args.no_cpu else 40) + (0 if args.no_extra else 80)
    budget_end = args.budget - legs_s
    log(f"workload built ({args.layout} layout); batched run until {budget_end:.0f} s")

    dt, steps, prof, st, pf, warm_s = run_batched(args, circ, budget_end)
    shots = steps * args.batch
    shots_per_s = shots / dt
    value = shots_per_s * ops

    # roofline of the kernel class that took the most time; achieved =
    # algorithmic flops ledgered from the actual (unpadded) dimensions of
    # every row / the class's summed launch durations (HIP events)
    total_ms = max(sum(v["ms"] for v in prof.values()), 1e-9)
    classes = {}
    for k, (bound, peak) in BOUND_OF.items():
        v = prof[k]
        sec = max(v["ms"] / 1e3, 1e-12)
        ach = v["alg_flops"] / sec
        c = {"share": v["ms"] / total_ms, "launches": v["launches"], "avg_ms": v["ms"] / max(v["launches"], 1),
             "achieved_tflops": ach / 1e12, "frac_of_flop_peak": ach / peak, "bound": bound, "frac": ach / peak}
        if v.get("alg_bytes"):
            ai = v["alg_flops"] / v["alg_bytes"]
            c["flops_per_byte"] = ai
            c["achieved_tbs"] = v["alg_bytes"] / sec / 1e12
            c["frac_of_hbm_peak"] = v["alg_bytes"] / sec / PEAK["hbm"]
            if ai < RIDGE.get(k, 0.0):
                c["bound"], c["frac"] = "hbm", c["frac_of_hbm_peak"]
        # flops the launches executed on their padded shapes (the statistics
        # run's count against one run's share of the time)
        padded = {"contract": st.get("gemm_flops"), "gram": st.get("gram_flops")}.get(k)
        if padded:
            c["executed_tflops"] = padded / max(v["ms"] / 1e3 / max(steps, 1), 1e-12) / 1e12
        classes[k] = c
    dom = max(BOUND_OF, key=lambda k: prof[k]["ms"])
    d, cd = prof[dom], classes[dom]
    sec = max(d["ms"] / 1e3, 1e-12)
    traffic = class_traffic(dom, args.batch, args.layout)
    per_launch = max(d["launches"], 1)
    if cd["bound"] == "hbm":
        roof = {"bound": "hbm", "achieved": d["alg_bytes"] / sec / 1e9, "peak": PEAK["hbm"] / 1e9,
                "unit": "GB/s", "frac": cd["frac"], "alg_bytes_per_launch": d["alg_bytes"] / per_launch,
                "per_unit": PER_UNIT_BYTES[dom], "flops_per_byte": cd["flops_per_byte"],
                "achieved_tflops": cd["achieved_tflops"], "frac_of_flop_peak": cd["frac_of_flop_peak"]}
    else:
        roof = {"bound": cd["bound"], "achieved": cd["achieved_tflops"], "peak": BOUND_OF[dom][1] / 1e12,
                "unit": "TFLOP/s", "frac": cd["frac"], "alg_flops_per_launch": d["alg_flops"] / per_launch,
                "per_unit": PER_UNIT["eigh" if dom.startswith("eigh") else dom]}
    roof.update({"traffic": traffic, "kernel_class": dom, "launches": d["launches"], "avg_ms": cd["avg_ms"],
                 "share_of_gpu_time": cd["share"]})
    if traffic is not None:
        roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 PMC, " + TRAFFIC["profile"] + ")"
        roof["traffic_rate_tbs"] = traffic / (roof["avg_ms"] / 1e3) / 1e12

    plain = None
    if not args.no_plain and elapsed() < args.budget - 60:
        sec, per_theta = run_plain(args, circ)
        plain = {"dtype": "c128", "batch": 1, "s_per_shot": sec, "shots_per_s": 1.0 / sec,
                 "trajectory_gates_per_s": ops / sec, "shots": args.plain_shots,
                 "s_per_shot_by_theta": per_theta}
        log(f"plain c128: {sec:.3f} s/shot")
    cpu = None
    if not args.no_cpu and elapsed() < args.budget - 45:
        rate, wall, (k0, k1) = cpu_oracle(circ, args.seed)
        model, nproc = host_cpu()
        cpu = {"value": rate, "unit": "trajectory-gates/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 lazy-ancilla state-vector oracle (numpy, 1 thread): ops {k0}-{k1} of one "
                         "d=5 C=5 SRX trajectory of the same op list, on the full 28-qubit live register, "
                         f"timed as the difference of two runs from the start ({wall:.1f} s of CPU work)",
               "host_cpu": model, "host_nproc": nproc}
        log(f"cpu oracle: {rate:.3f} trajectory-gates/s")
    other = grad = graph = None
    if not args.no_extra:
        if elapsed() < args.budget - 45:
            other = run_layout_leg(args, "default" if args.layout == "optimized" else "optimized", 1024)
            log(f"other layout: {other['shots_per_s']:.1f} shots/s")
        if elapsed() < args.budget - 15:
            grad = run_gradient(args)
            log(f"gradient: {grad['records_per_s']:.1f} records/s")
        if elapsed() < args.budget - 20:
            graph = run_graph_leg(args, circ, 256)
            log(f"run modes at B=256: {graph}")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "trajectory-gates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": dt / max(steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (FP32 MFMA) + f64 (Gram, eigen, probabilities)",
        "data": "synthetic",
        "config": {"workload": f"d=5 colour code, 37 qubits, {args.rounds} rounds, SRX theta grid "
                               "linspace(0.02,0.2,8), chi_max=64, cutoff 1e-10, batched complex64",
                   "batch": args.batch, "ops_per_shot": ops, "leaves": circ.n_leaves,
                   "layout": ("clustered (App. B, Algorithm 1)" if args.layout == "optimized"
                              else "default (qubit i on leaf i)"),
                   "parallelism": "single GPU"},
        "steps_requested": args.steps,
        "shots_per_s": shots_per_s,
        "roofline": roof,
        "cpu_baseline": cpu,
        "plain_c128": plain,
        "speedup_vs_plain_c128": (shots_per_s * plain["s_per_shot"]) if plain else None,
        "warmup_step_s": warm_s,
        "kernel_time_ms": {k: round(v["ms"], 3) for k, v in prof.items()},
        "kernel_classes": classes,
        "p_fail_by_theta": pf,
        "other_layout": other,
        "log_prob_grad": grad,
        "run_modes": graph,
        "run_stats": {"max_rank": st.get("max_rank"),
                      "mean_discarded_weight": (st["discarded_weight"] / args.batch
                                                if "discarded_weight" in st else None),
                      "degenerate_cuts_per_shot": (st["degenerate_cuts"] / args.batch
                                                   if "degenerate_cuts" in st else None),
                      "hops_per_batch": st.get("hops"), "block_hops_per_batch": st.get("block_hops"),
                      "launches_per_batch": st.get("launches"),
                      "engine_device_gib": st.get("engine_device_gib"),
                      "gemm_tile_autotune": st.get("autotune")},
        "wall_s": elapsed(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
