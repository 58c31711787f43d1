"""Benchmark: LLG spin-updates/s of the fused Depondt step on one MI355X.

Workload (default): triangular lattice 512 x 512 (262,144 spins), exchange
shells J1..J3 = 1, -0.2, -0.1 meV, interfacial DMI 0.2 meV, K = 0.05 meV,
B = 0.5 T, stochastic LLG at T = 10 K (Philox thermal field), alpha = 0.1,
dt = 0.5 fs, FP32 spins with FP64 observables every 100 steps.  A "step"
is one full Depondt step (predictor + corrector) of every spin.

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BYTES_PER_UPDATE = {"f32": 24.0, "f64": 48.0}   # read n, write n(t+dt): 3 components each


def cpu_baseline(workload, budget_s: float = 12.0) -> dict:
    """The FP64 oracle, as it stands, on the host cores: Depondt steps of the
    same workload until about budget_s seconds of CPU work have been spent."""
    import oracle
    import spin_inputs as si

    oracle.build(force=False)
    w = workload
    s = oracle.System(w.geometry, w.hamiltonian)
    n = si.uniform_sphere(s.N, w.init_seed)
    d = w.dynamics
    steps = 0
    t0 = time.perf_counter()
    while True:
        n, _ = s.run(n, d.alpha, d.dt, 1, T=d.T, seed=d.seed, step0=steps)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 2000:
            break
    return {"value": s.N * steps / el, "unit": "spin-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} FP64 Depondt steps of the full {s.N}-spin workload ({el:.1f} s)"}


def calibrate_copy(mib: int, reps: int = 5) -> None:
    """A plain device-to-device copy of known size: the reference that HBM
    byte counters (FETCH_SIZE / WRITE_SIZE) are scaled against."""
    import torch

    n = mib * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(json.dumps({"calibration": "copy", "bytes_read_per_launch": 4 * n,
                      "bytes_written_per_launch": 4 * n, "ms_per_launch": ms,
                      "GBps": 8 * n / (ms * 1e-3) / 1e9}), flush=True)


_STREAM = None


def work_stream():
    """One dedicated (non-default, default-priority) stream: the engines
    launch every kernel on it and the timing events are recorded on it."""
    global _STREAM
    import torch

    if _STREAM is None:
        _STREAM = torch.cuda.Stream()
        assert _STREAM.cuda_stream != 0
    return _STREAM


def bench_batch(args) -> dict:
    """96 replicas (sides from {32, 64, 128, 256}, T uniform in 0-100 K, the
    square32 Hamiltonian, FP32) advanced as one batch, against the same
    replicas advanced one engine at a time."""
    import torch

    import paper_1901_11350_amd as pk
    import spin_inputs as si
    from spin_inputs.workloads import batch_replica_table

    table = batch_replica_table(96, 11353)
    ham = si.WORKLOADS["square32_fp64"].hamiltonian
    alpha, dt, seed = 0.3, 0.001, 11353
    stream = work_stream()
    b = pk.Batch(0, stream=stream)
    engines = []
    for r, (L, T) in enumerate(table):
        e = pk.Engine(0, "f32", stream=stream)
        e.set_geometry(si.square(L, L))
        e.set_hamiltonian(ham)
        e.set_spins(si.uniform_sphere(e.N, 20000 + r))
        b.add(e, alpha, dt, T=T, seed=seed, replica=r)
        engines.append((e, T, r))
    total = sum(L * L for L, _ in table)
    b.set_chunk(args.batch_chunk)
    tuned = b.autotune(8)
    b.run(args.batch_chunk)
    torch.cuda.synchronize()
    K = args.batch_steps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    b.run(K)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    # the same replicas, one engine (one launch per step each) at a time
    Ks = max(10, K // 10)
    for e, T, r in engines:
        e.run(alpha, dt, 2, T=T, seed=seed, replica=r)
    torch.cuda.synchronize()
    ev0.record(stream)
    for e, T, r in engines:
        e.run(alpha, dt, Ks, T=T, seed=seed, replica=r)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_sep = ev0.elapsed_time(ev1)
    n_res = sum(1 for r in range(len(table)) if b.info(r)[1])
    return {"workload": "batch96_square", "replicas": len(table), "resident_replicas": n_res,
            "total_spins": total, "steps": K, "chunk": args.batch_chunk,
            "spin_updates_per_s": total * K / (ms * 1e-3), "ms_per_step": ms / K,
            "separate_engines_spin_updates_per_s": total * Ks / (ms_sep * 1e-3),
            "batch_gain": (total * K / ms) / (total * Ks / ms_sep), "autotune_ms_per_step": tuned}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", action="store_true",
                    help="also time the 96-replica batch (reported under 'batch')")
    ap.add_argument("--batch-steps", type=int, default=256)
    ap.add_argument("--batch-chunk", type=int, default=32)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="only run a device copy of this size (counter calibration)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="triangular512_sllg")
    ap.add_argument("--observe-every", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1901_11350_amd as pk
    import spin_inputs as si

    w = si.WORKLOADS[args.workload]
    d = w.dynamics
    torch.cuda.init()
    stream = work_stream()
    e = pk.engine_for(w, 0, w.precision, stream=stream)
    if w.init == "conical_helix":
        n0 = si.conical_helix(w.geometry, seed=w.init_seed)
    else:
        n0 = si.uniform_sphere(e.N, w.init_seed)
    e.set_spins(n0)
    tuned_ms = None
    if not args.no_autotune:
        tuned_ms = e.autotune(d.alpha, d.dt, d.T, d.seed, n_steps=50)
    print(f"[bench] workload={w.name} N={e.N} path={e.step_path} precision={w.precision} "
          f"autotune_ms={tuned_ms}", file=sys.stderr, flush=True)

    # warm-up
    e.run(d.alpha, d.dt, args.warmup, T=d.T, seed=d.seed)
    torch.cuda.synchronize()

    # timed: full runs with observables (the benchmark value)
    K = args.steps
    oe = args.observe_every if args.observe_every and K >= args.observe_every else 0
    t_ev0 = torch.cuda.Event(enable_timing=True)
    t_ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_ev0.record(stream)
    obs = e.run(d.alpha, d.dt, K, T=d.T, seed=d.seed, observe_every=oe)
    t_ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t_ev0.elapsed_time(t_ev1)
    value = e.N * K / (ms * 1e-3)

    # dominant kernel: the step kernel alone (no observables), per launch
    K2 = max(100, K // 2)
    k_ev0 = torch.cuda.Event(enable_timing=True)
    k_ev1 = torch.cuda.Event(enable_timing=True)
    k_ev0.record(stream)
    e.run(d.alpha, d.dt, K2, T=d.T, seed=d.seed)
    k_ev1.record(stream)
    torch.cuda.synchronize()
    launches_per_step = 2 if e.step_path == "twopass" else 1
    t_launch = k_ev0.elapsed_time(k_ev1) * 1e-3 / (K2 * launches_per_step)
    bytes_per_launch = BYTES_PER_UPDATE[w.precision] * e.N / launches_per_step
    achieved = bytes_per_launch / t_launch / 1e9

    last = obs[-1] if obs else e.observe()
    line = {
        "metric": "LLG spin-updates/s at 1 GPU + HBM GB/s; surrogate vs direct dipole speedup at 1e-3",
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.precision,
        "data": "synthetic",
        "config": {"workload": w.name, "n_sites": e.N, "lattice": w.description,
                   "alpha": d.alpha, "dt_ps": d.dt, "T_K": d.T, "observe_every": oe,
                   "step_path": e.step_path},
        "hbm_gbps_algorithmic": value * BYTES_PER_UPDATE[w.precision] / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": {"fused2d": "k_depondt_fused2d", "twopass": "k_predict+k_correct"}.get(
                         e.step_path, "k_fused2d_shape"),
                     "bytes_per_launch": bytes_per_launch, "us_per_launch": t_launch * 1e6},
        "wall_s": wall,
        "final_observation": {"E_per_spin": last["E"] / e.N, "max_norm_dev": last["max_norm_dev"]},
    }
    if args.batch:
        line["batch"] = bench_batch(args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
