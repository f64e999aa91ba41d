"""Write the oracle's ensemble statistics used by tests/test_gpu_ensemble.py.

    python tests/golden/make_ensemble.py        # ~25 min of CPU, 8 processes

Calls only the FP64 oracle (oracle/) and the seeded input generator: eight
random quenches (phi0 uniform in +-0.05, seeds 700 .. 707, omega0 = 0) of the
inertial model on a 128 x 128 grid (spacing 1, A = B = kappa = M = eta =
rho = 1, gdot = 0.05, dt = 0.005), 20000 steps each (t = 100, strain 5: five
strain wraps), sampled every 2000 steps: L_s, L_par, L_perp, sigma_xy,
sigma_xy_re and the S(k) shells.  Output: ensemble_128.json beside this file.
"""
from __future__ import annotations

import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N, GDOT, STEPS, EVERY, SEEDS = 128, 0.05, 20000, 2000, tuple(range(700, 708))
PARAMS = dict(nx=N, ny=N, lx=float(N), ly=float(N), gdot=GDOT, A=1.0, B=1.0, kappa=1.0,
              M=1.0, eta=1.0, rho=1.0, dt=0.005)


def one(seed):
    from oracle import model_h as mh
    from oracle import observables as ob
    from paper_0710_5912_amd import inputs

    p = mh.Params(**PARAMS)
    st = mh.initial_state(p, inputs.noise_phi0(N, N, seed, amp=0.05))
    rows = []
    for _ in range(STEPS // EVERY):
        st = mh.run(p, st, EVERY)
        o, sk, _ = ob.observables(p, st)
        rows.append(dict(step=st.step, Ls=o["Ls"], L_par=o["L_par"], L_perp=o["L_perp"],
                         sigma_xy=o["sigma_xy"], sigma_xy_re=o["sigma_xy_re"],
                         mean_phi=o["mean_phi"], Sk=[float(v) for v in sk]))
    return seed, rows


def main():
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        runs = dict(ex.map(one, SEEDS))
    out = dict(params=PARAMS, steps=STEPS, every=EVERY, seeds=list(SEEDS), amp=0.05,
               runs={str(s): runs[s] for s in SEEDS})
    with open(os.path.join(HERE, "ensemble_128.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
