"""Writes mc_sc_ferromagnet_oracle_stats.json: equilibrium statistics of the
simple-cubic Heisenberg ferromagnet (J = 1 meV, mu = 2, no field, periodic
L^3) from the oracle's Metropolis sweeps (Sec. III.B: every spin once per
sweep, sequentially in random order; adaptive cone during thermalisation).

Protocol for each (L, T): start from the ferromagnet along +z; 4,000
thermalisation sweeps with the adaptive cone (initial 60 degrees, target
acceptance 0.5); then SAMPLES sweeps at the cone the feedback reached,
one observation per sweep.  Reported: <E>/N, <|M|> (M = mean spin) and the
Binder cumulant U4 = 1 - <m^4> / (3 <m^2>^2), each with the standard error
from BLOCKS blocks of consecutive sweeps (U4 by jackknife over the blocks).

Calls only the oracle; run from the repository root:
    python tests/golden/make_mc_stats.py
"""

import json
import math
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

SIZES = (8, 12)
TEMPS = (14.0, 16.7, 20.0)
THERM = 4000
SAMPLES = 200000
BLOCKS = 50
CONE0 = 60.0
TARGET = 0.5
SEED = 31


def block_stats(E, m, blocks):
    """Means and blocked standard errors of E/N and |M|, and U4 with its
    jackknife error over the blocks."""
    nb = len(E) // blocks
    E = E[: nb * blocks].reshape(blocks, nb)
    m = m[: nb * blocks].reshape(blocks, nb)
    eb, mb = E.mean(axis=1), m.mean(axis=1)
    m2b, m4b = (m ** 2).mean(axis=1), (m ** 4).mean(axis=1)

    def u4(m2, m4):
        return 1.0 - m4 / (3.0 * m2 * m2)

    u = u4(m2b.mean(), m4b.mean())
    jk = np.array([u4(np.delete(m2b, k).mean(), np.delete(m4b, k).mean()) for k in range(blocks)])
    u_err = math.sqrt((blocks - 1) / blocks * ((jk - jk.mean()) ** 2).sum())
    return {"E_per_spin": float(eb.mean()), "E_per_spin_err": float(eb.std(ddof=1) / math.sqrt(blocks)),
            "M_abs": float(mb.mean()), "M_abs_err": float(mb.std(ddof=1) / math.sqrt(blocks)),
            "U4": float(u), "U4_err": float(u_err)}


def one(args):
    L, T = args
    import oracle
    import spin_inputs as si

    oracle.build(force=False)
    oracle.set_num_threads(1)
    ham = si.Hamiltonian(mu=(2.0,), B=(0, 0, 0), K=(0.0,), K_axis=((0, 0, 1),), J=(1.0,))
    s = oracle.System(si.simple_cubic(L, L, L), ham)
    n, _, _, cone = s.mc_run(si.ferromagnet(s.N, (0, 0, 1)), T, CONE0, THERM, seed=SEED,
                             target_acceptance=TARGET, return_cone=True)
    n, obs, acc = s.mc_run(n, T, cone, SAMPLES, seed=SEED, sweep0=THERM, observe_every=1)
    E = np.array([o["E"] for o in obs]) / s.N
    m = np.array([np.linalg.norm(o["M"]) for o in obs])
    out = block_stats(E, m, BLOCKS)
    out.update({"L": L, "T_K": T, "cone_deg": cone, "acceptance": acc / (SAMPLES * s.N)})
    return out


def main():
    cases = [(L, T) for L in SIZES for T in TEMPS]
    with ProcessPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        res = list(ex.map(one, cases))
    doc = {"what": "oracle Metropolis statistics of the simple-cubic ferromagnet (J = 1 meV, mu = 2, B = 0, "
                   "periodic L^3); see make_mc_stats.py for the protocol",
           "thermalisation_sweeps": THERM, "samples": SAMPLES, "blocks": BLOCKS, "cone0_deg": CONE0,
           "target_acceptance": TARGET, "seed": SEED, "results": res}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "mc_sc_ferromagnet_oracle_stats.json"),
              "w") as f:
        json.dump(doc, f, indent=1)
    for r in res:
        print(r)


if __name__ == "__main__":
    main()
