"""Writes mc_lattices_oracle_stats.json: equilibrium statistics from the
oracle's Metropolis sweeps (Sec. III.B: every spin once per sweep,
sequentially in random order; adaptive cone during thermalisation) on
lattices whose bonds need more than two colours in a parallel sweep: the
triangular lattice (nearest neighbours), the honeycomb lattice (two atoms,
first and second shells) and the kagome lattice (three atoms).

Protocol for each case: start from the ferromagnet along +z; THERM
thermalisation sweeps with the adaptive cone (initial 60 degrees, target
acceptance 0.5); then SAMPLES sweeps at the cone the feedback reached, one
observation per sweep.  Reported: <E>/N, <|M|> and U4 with blocked standard
errors (make_mc_stats.block_stats).

Calls only the oracle; run from the repository root:
    python tests/golden/make_mc_stats_lattices.py
"""

import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

THERM = 4000
SAMPLES = 100000
BLOCKS = 50
CONE0 = 60.0
TARGET = 0.5
SEED = 47


def lattice_cases():
    """name -> (geometry, Hamiltonian, temperatures)."""
    import spin_inputs as si

    return {
        "triangular12x12": (si.triangular(12, 12),
                            si.Hamiltonian(mu=(2.0,), B=(0, 0, 0), K=(0.1,), K_axis=((0, 0, 1),), J=(1.0,)),
                            (5.0, 12.0)),
        "honeycomb8x8_2shell": (si.honeycomb(8, 8),
                                si.Hamiltonian(mu=(2.0, 2.0), B=(0, 0, 0), K=(0.05, 0.05),
                                               K_axis=((0, 0, 1), (0, 0, 1)), J=(1.0, 0.3)),
                                (5.0, 12.0)),
        "kagome6x6": (si.kagome(6, 6),
                      si.Hamiltonian(mu=(2.0, 2.0, 2.0), B=(0, 0, 0.5), K=(0.0, 0.0, 0.0),
                                     K_axis=((0, 0, 1),) * 3, J=(1.0,)),
                      (4.0,)),
    }


def one(args):
    name, T = args
    import oracle
    import spin_inputs as si
    from make_mc_stats import block_stats

    oracle.build(force=False)
    oracle.set_num_threads(1)
    geo, ham, _ = lattice_cases()[name]
    s = oracle.System(geo, ham)
    n, _, _, cone = s.mc_run(si.ferromagnet(s.N, (0, 0, 1)), T, CONE0, THERM, seed=SEED,
                             target_acceptance=TARGET, return_cone=True)
    n, obs, acc = s.mc_run(n, T, cone, SAMPLES, seed=SEED, sweep0=THERM, observe_every=1)
    E = np.array([o["E"] for o in obs]) / s.N
    m = np.array([np.linalg.norm(o["M"]) for o in obs])
    out = block_stats(E, m, BLOCKS)
    out.update({"case": name, "T_K": T, "cone_deg": cone, "acceptance": acc / (SAMPLES * s.N)})
    return out


def main():
    cases = [(name, T) for name, (_, _, temps) in lattice_cases().items() for T in temps]
    with ProcessPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        res = list(ex.map(one, cases))
    doc = {"what": "oracle Metropolis statistics on triangular, honeycomb and kagome lattices; see "
                   "make_mc_stats_lattices.py for the cases and the protocol",
           "thermalisation_sweeps": THERM, "samples": SAMPLES, "blocks": BLOCKS, "cone0_deg": CONE0,
           "target_acceptance": TARGET, "seed": SEED, "results": res}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "mc_lattices_oracle_stats.json"), "w") as f:
        json.dump(doc, f, indent=1)
    for r in res:
        print(r)


if __name__ == "__main__":
    main()
