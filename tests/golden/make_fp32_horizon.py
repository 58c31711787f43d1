"""Writes fp32_horizon.json: the trajectory-parity horizon of the FP32 path
(the last step at which two FP64 oracle runs whose initial states differ by
about 1e-7 per component still agree within 1e-5 in every spin component),
for the stochastic 512^2 triangular workload (T = 10 K, the same Philox
stream in both runs) and the 128^3 simple-cubic workload (T = 0), and the
oracle's energy per spin and mean spin every 100 steps of both runs over
each workload's full step count (the statistics compared beyond the
horizon, with the two runs' own difference as their scale).

Calls only the oracle; run from the repository root:
    python tests/golden/make_fp32_horizon.py [workload ...]
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

PERTURB = 1e-7
BAR = 1e-5
CHUNK = 5
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp32_horizon.json")


def initial(w):
    import spin_inputs as si

    if w.init == "conical_helix":
        return si.conical_helix(w.geometry, seed=w.init_seed)
    return si.uniform_sphere(w.geometry.n_sites, w.init_seed)


def perturbed(n, seed=7):
    g = np.random.default_rng(seed).standard_normal(n.shape)
    m = n + PERTURB * g
    return m / np.linalg.norm(m, axis=0)


def horizon(name):
    import oracle
    import spin_inputs as si

    oracle.build(force=False)
    w = si.WORKLOADS[name]
    d = w.dynamics
    s = oracle.System(w.geometry, w.hamiltonian)
    a = initial(w)
    b = perturbed(a)
    dev0 = float(np.abs(a - b).max())
    H = None
    curve = []
    obs_a, obs_b = [], []
    t0 = time.time()
    for step in range(0, d.n_steps, CHUNK):
        a, oa = s.run(a, d.alpha, d.dt, CHUNK, T=d.T, seed=d.seed, step0=step)
        b, ob = s.run(b, d.alpha, d.dt, CHUNK, T=d.T, seed=d.seed, step0=step)
        k = step + CHUNK
        dev = float(np.abs(a - b).max())
        curve.append((k, dev))
        if H is None and dev > BAR:
            H = k - CHUNK
        if k % d.observe_every == 0:
            for n, acc in ((a, obs_a), (b, obs_b)):
                o = s.observe(n, k)
                acc.append({"step": k, "E_per_spin": o["E"] / s.N, "M": list(o["M"])})
        if k % 500 == 0:
            print(f"[{name}] step {k}: max deviation {dev:.3e} ({time.time() - t0:.0f} s)", flush=True)
    return {"workload": name, "n_sites": s.N, "steps": d.n_steps, "initial_deviation": dev0,
            "bar": BAR, "horizon": H if H is not None else d.n_steps, "horizon_reached": H is not None,
            "max_deviation_every_step_chunk": curve[:: max(1, len(curve) // 200)],
            "observations_run": obs_a, "observations_perturbed": obs_b}


def main():
    names = sys.argv[1:] or ["triangular512_sllg", "cubic128_bulkdmi"]
    doc = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            doc = json.load(f)
    for name in names:
        doc[name] = horizon(name)
        with open(OUT, "w") as f:
            json.dump(doc, f, indent=0)
        print(name, "horizon", doc[name]["horizon"], flush=True)


if __name__ == "__main__":
    main()
