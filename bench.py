#!/usr/bin/env python3
"""Throughput of the TTN trajectory engine on one MI355X.

Workload: the d=5 triangular colour code (37 qubits: 19 data + 18 ancillas),
5 rounds of X-then-Z syndrome extraction, a systematic X over-rotation
exp(-i theta X / 2) after every gate, initialisation and idle location with
theta cycling over an 8-point grid in [0.02, 0.2] rad across trajectories,
binary tree over 64 leaves (default qubit-to-leaf order), chi_max = 64,
squared-weight cutoff 1e-10; contractions in complex64 on FP32 MFMA,
Gram matrices / eigen-decompositions / probabilities in FP64.

A step is one batched run of the whole circuit (2427 ops per trajectory:
CNOTs, noise ops, initialisations, measurements) for `--batch` trajectories.
The metric is trajectory-gates/s = trajectories/s x ops per trajectory; the
same run in complex128, one trajectory at a time (the plain path), and the
FP64 CPU oracle on a bounded sample are reported beside it.  Extra legs: the
same workload with the clustered qubit-to-leaf layout (App. B), and log P
with its adjoint gradient for records of the differentiation workload.

Prints one JSON line.  --gpus N > 1 is not supported (one GPU per box).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "trajectory-gates/s and shots/s at d=5 chi=64, batched cplx64 vs plain cplx128"
PEAK = {"fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "fp64_valu": 78.6e12, "hbm": 8.0e12}
THETAS = [0.02 + i * (0.2 - 0.02) / 7 for i in range(8)]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def theta_rows(circ, rows, offset):
    import numpy as np
    th = np.asarray(THETAS)[(offset + np.arange(rows)) % len(THETAS)]
    return np.repeat(th[:, None], circ.n_loc, axis=1)


def run_batched(args, circ):
    import numpy as np
    import torch
    from paper_2511_05719_amd import TTNEngine
    B = args.batch
    free0, _ = torch.cuda.mem_get_info()
    eng = TTNEngine(circ.n_qubits, B, circ.leaf_of_qubit, chi_max=64, cutoff=1e-10, dtype="c64",
                    seed=args.seed)
    free1, _ = torch.cuda.mem_get_info()
    ol = eng.upload(circ)
    # GEMM tile shapes measured during the warm-up (the timed steps reuse
    # the choices and measure nothing)
    eng.autotune(not args.no_autotune and args.warmup > 0)
    for w in range(args.warmup):
        eng.run_circuit(ol, theta=theta_rows(circ, B, w * B), traj_offset=w * B, stats=False)
        torch.cuda.synchronize()
        log(f"warmup step {w} done")
    tuned = eng.autotune(False)
    params = [theta_rows(circ, B, (args.warmup + k) * B) for k in range(args.steps)]
    params_dev = [torch.as_tensor(p, device="cuda") for p in params]
    eng.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for k in range(args.steps):
        res = eng.run_circuit(ol, theta=params_dev[k], traj_offset=(args.warmup + k) * B, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = eng.profile_read()
    eng.profile(False)
    log(f"timed {args.steps} steps in {t1 - t0:.3f} s")
    # one more step with statistics (untimed) for the report
    st = eng.run_circuit(ol, theta=params_dev[0], traj_offset=args.warmup * B, stats=True).stats
    fail = eng.decode(res.records, circ.data_rec, circ.code.checks)
    p_fail = float(fail.float().mean().item())
    eng.close()
    st["engine_device_gib"] = (free0 - free1) / 2 ** 30
    st["autotune"] = {"shapes_measured": tuned[0], "differs_from_fixed_rule": tuned[1]}
    return t1 - t0, prof, st, p_fail


def run_plain(args, circ):
    import torch
    from paper_2511_05719_amd import TTNEngine
    eng = TTNEngine(circ.n_qubits, 1, circ.leaf_of_qubit, chi_max=64, cutoff=1e-10, dtype="c128",
                    seed=args.seed)
    ol = eng.upload(circ)
    eng.run_circuit(ol, theta=theta_rows(circ, 1, 0), traj_offset=0, stats=False)   # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.plain_shots):
        eng.run_circuit(ol, theta=theta_rows(circ, 1, 3 * i + 1), traj_offset=3 * i + 1, stats=False)
        torch.cuda.synchronize()
    t1 = time.perf_counter()
    eng.close()
    return (t1 - t0) / args.plain_shots


def run_optimized(args):
    """The same workload with the clustered qubit-to-leaf layout (App. B)."""
    import torch
    from paper_2511_05719_amd import TTNEngine
    from workload import build_circuit, exact_bond_dim
    circ = build_circuit(5, args.rounds, "srx", leaf_of_qubit="optimized")
    B = args.batch
    eng = TTNEngine(circ.n_qubits, B, circ.leaf_of_qubit, chi_max=64, cutoff=1e-10, dtype="c64", seed=args.seed)
    ol = eng.upload(circ)
    eng.autotune(not args.no_autotune)
    eng.run_circuit(ol, theta=theta_rows(circ, B, 0), traj_offset=0, stats=False)
    torch.cuda.synchronize()
    eng.autotune(False)
    steps = 2
    t0 = time.perf_counter()
    for k in range(steps):
        res = eng.run_circuit(ol, theta=theta_rows(circ, B, (k + 1) * B), traj_offset=(k + 1) * B, stats=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = eng.run_circuit(ol, theta=theta_rows(circ, B, B), traj_offset=B, stats=True).stats
    p_fail = float(eng.decode(res.records, circ.data_rec, circ.code.checks).float().mean().item())
    eng.close()
    shots = steps * B / dt
    return {"layout": "clustered (App. B, Algorithm 1)", "batch": B, "steps": steps,
            "shots_per_s": shots, "trajectory_gates_per_s": shots * circ.n_ops,
            "chi_exact_clifford_skeleton": exact_bond_dim(build_circuit(5, args.rounds, "none",
                                                                        leaf_of_qubit=circ.leaf_of_qubit).ops,
                                                          circ.n_qubits, circ.leaf_of_qubit),
            "p_fail": p_fail, "mean_discarded_weight": st.get("discarded_weight", 0.0) / B,
            "max_rank": st.get("max_rank")}


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


def cpu_oracle(circ, seed):
    """The FP64 oracle (lazy-ancilla state vector, numpy, one thread) on the
    same circuit: ops 47-54 of one trajectory, all on the full 28-qubit live
    register, timed as the difference of two runs."""
    import numpy as np
    from oracle import statevector as sv
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:
        lim = None
    ka, kb = 46, 54
    t0 = time.perf_counter()
    sv.run(circ, 0.1, 0.0, seed, np.arange(1), stop_after_op=ka)
    t1 = time.perf_counter()
    sv.run(circ, 0.1, 0.0, seed, np.arange(1), stop_after_op=kb)
    t2 = time.perf_counter()
    if lim is not None:
        lim.unregister() if hasattr(lim, "unregister") else None
    rate = (kb - ka) / max((t2 - t1) - (t1 - t0), 1e-9)
    return rate, (t2 - t0)


# HBM traffic of one launch of a kernel class at this workload and B=3072
# (rocprofv3 FETCH_SIZE / WRITE_SIZE passes, each scaled by what the counter
# reads for a 256 MiB device copy, see the profile named), valid for the
# source file it was measured on: reported only while that file is unchanged
TRAFFIC = {
    "profile": "profiles/ttn_d5_chi64_b3072_hbm_traffic.txt",
    "batch": 3072,
    "classes": {
        # k_zgemm<float2, float2, float2, ...>, all tile shapes
        "contract": {"bytes_per_launch": 1.766e9, "source": "ttn_gemm.hip",
                     "sha256": "df0e24b983f08d00be0362e823a71c7ab335629e54e886fbf60a46ef502d37b8"},
        # k_zgemm<float2, float2, double2, ...>, all tile shapes
        "gram": {"bytes_per_launch": 0.7721e9, "source": "ttn_gemm.hip",
                 "sha256": "df0e24b983f08d00be0362e823a71c7ab335629e54e886fbf60a46ef502d37b8"},
        # k_jacobi<false, ...> + k_jacobi_coset<128> + k_jacobi_vectors<128> per launch
        "eigh_large": {"bytes_per_launch": 11.656e9, "source": "ttn_eigh.hip",
                       "sha256": "b7089238a01ebf7eb10ab9b6c5bbe7cf18b1da0d839904710c3ec621df88a52c"},
    },
}


def class_traffic(cls, batch):
    import hashlib
    ent = TRAFFIC["classes"].get(cls)
    if ent is None or batch != TRAFFIC["batch"]:
        return None
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2511_05719_amd", "csrc", ent["source"])
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=3072)
    ap.add_argument("--rounds", type=int, default=5)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--plain-shots", type=int, default=4)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the clustered-layout and gradient legs")
    ap.add_argument("--no-autotune", action="store_true", help="fixed-rule GEMM tile shapes (no measuring "
                    "in the warm-up)")
    ap.add_argument("--grad-records", type=int, default=64)
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
    circ = build_circuit(5, args.rounds, "srx")
    ops = ops_per_shot(circ)

    dt, prof, st, p_fail = run_batched(args, circ)
    shots = args.steps * args.batch
    shots_per_s = shots / dt
    value = shots_per_s * ops

    # roofline of the kernel class that took the most time; achieved =
    # algorithmic flops ledgered from the actual (unpadded) dimensions of
    # every row / the class's summed launch durations (HIP events)
    per_unit = {
        "eigh": "36 n^3 real flops per n x n complex Hermitian eigen-decomposition with vectors, "
                "n = actual bond dimension (non-zero Gram eigenvalues)",
        "gram": "8 n^2 r real flops per Gram matrix (n = actual bond dimension, r = product of the other "
                "two actual leg dimensions; per diagonal block in block-diagonal moves)",
        "contract": "8 k n r real flops per factor product (k kept, n actual bond dimension, r = product "
                    "of the other two actual leg dimensions)",
        "move": "8 (r^2 (3n - 2r) / 3 + r^3 / 3) real flops per exact centre move (pivoted Cholesky of "
                "rank r and the inverse of its triangle, n = problem size)",
    }
    bound_of = {"contract": ("mfma", PEAK["fp32_mfma"]), "gram": ("mfma", PEAK["fp64_mfma"]),
                "eigh_small": ("alu", PEAK["fp64_valu"]), "eigh_large": ("alu", PEAK["fp64_valu"]),
                "move": ("alu", PEAK["fp64_valu"])}
    total_ms = max(sum(v["ms"] for v in prof.values()), 1e-9)
    classes = {}
    for k, (bound, peak) in bound_of.items():
        v = prof[k]
        ach = v["alg_flops"] / max(v["ms"] / 1e3, 1e-12)
        classes[k] = {"share": v["ms"] / total_ms, "launches": v["launches"],
                      "avg_ms": v["ms"] / max(v["launches"], 1), "achieved_tflops": ach / 1e12,
                      "frac": ach / peak, "bound": bound}
        # flops the launches executed on their padded shapes (one run's
        # count from the statistics run, against one run's share of the time)
        padded = {"contract": st.get("gemm_flops"), "gram": st.get("gram_flops")}.get(k)
        if padded:
            classes[k]["executed_tflops"] = padded / max(v["ms"] / 1e3 / args.steps, 1e-12) / 1e12
    dom = max(bound_of, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    bound, peak = bound_of[dom]
    achieved = d["alg_flops"] / max(d["ms"] / 1e3, 1e-12)
    traffic = class_traffic(dom, args.batch)
    roof = {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic, "kernel_class": dom, "launches": d["launches"],
            "avg_ms": d["ms"] / max(d["launches"], 1), "share_of_gpu_time": d["ms"] / total_ms,
            "per_unit": per_unit["eigh" if dom.startswith("eigh") else dom]}
    if traffic is not None:
        roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 PMC, " + TRAFFIC["profile"] + ")"
        roof["traffic_rate_tbs"] = traffic / (roof["avg_ms"] / 1e3) / 1e12

    plain = None
    if not args.no_plain:
        sec = run_plain(args, circ)
        plain = {"dtype": "c128", "batch": 1, "s_per_shot": sec, "shots_per_s": 1.0 / sec,
                 "trajectory_gates_per_s": ops / sec, "shots": args.plain_shots}
    optimized = grad = None
    if not args.no_extra:
        optimized = run_optimized(args)
        log(f"clustered layout: {optimized['shots_per_s']:.1f} shots/s")
        grad = run_gradient(args)
        log(f"gradient: {grad['records_per_s']:.1f} records/s")
    cpu = None
    if not args.no_cpu:
        rate, wall = cpu_oracle(circ, args.seed)
        cpu = {"value": rate, "unit": "trajectory-gates/s", "cores": 1, "kind": "oracle",
               "sample": "FP64 lazy-ancilla state-vector oracle (numpy, 1 thread): ops 47-54 of one "
                         "d=5 C=5 SRX trajectory on the full 28-qubit live register "
                         f"({wall:.1f} s of CPU work)"}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "trajectory-gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (FP32 MFMA) + f64 (Gram, eigen, probabilities)",
        "data": "synthetic",
        "config": {"workload": f"d=5 colour code, 37 qubits, {args.rounds} rounds, SRX theta grid "
                               "linspace(0.02,0.2,8), chi_max=64, cutoff 1e-10, batched complex64",
                   "batch": args.batch, "ops_per_shot": ops, "leaves": circ.n_leaves,
                   "layout": "default (qubit i on leaf i)", "parallelism": "single GPU"},
        "shots_per_s": shots_per_s,
        "roofline": roof,
        "cpu_baseline": cpu,
        "plain_c128": plain,
        "speedup_vs_plain_c128": (shots_per_s * plain["s_per_shot"]) if plain else None,
        "kernel_time_ms": {k: round(v["ms"], 3) for k, v in prof.items()},
        "kernel_classes": classes,
        "clustered_layout": optimized,
        "log_prob_grad": grad,
        "run_stats": {"p_fail": p_fail, "max_rank": st.get("max_rank"),
                      "mean_discarded_weight": st.get("discarded_weight", 0.0) / args.batch,
                      "hops_per_batch": st.get("hops"), "block_hops_per_batch": st.get("block_hops"),
                      "launches_per_batch": st.get("launches"),
                      "engine_device_gib": st.get("engine_device_gib"),
                      "gemm_tile_autotune": st.get("autotune")},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
