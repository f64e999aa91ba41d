"""The Table I campaigns as commands (one JSON line per set, then a summary).

  python -m paper_0710_5912_amd.campaigns dv-sheared   [--strain 80] [--samples 100] [--refine 2] [--sets DV5s,DV6s]
  python -m paper_0710_5912_amd.campaigns zero-shear   [--seeds 4] [--refine 2] [--sets DV6u]
  python -m paper_0710_5912_amd.campaigns steady-states [--strain 150] [--lb-sets] [--refine 2] [--sets R030s]

dv-sheared: the inertialess sheared sets DV1s .. DV6s, L_par and L_perp
against strain (Section VIII D).  zero-shear: the sets DV1u .. DV6u and
R028u .. R032u to L_s = 0.025, growth exponents of L_s(t) by the protocol of
Section VIII A with a fitted offset.  --refine 2 runs the sets on a grid of
half the mesh interval at the same interfacial width (the low-viscosity DV sets
need it: on the Table I grid, l = 0.8 mesh intervals, they become non-finite).  steady-states: the inertial sheared
sets of the scaling plot to the given strain, averages over strain >= 100
and the power-law fits of L_par, L_perp against gdot t_VI (Section VIII B);
with --lb-sets the sets R028s, R022s, R029s of Table I, averages only.
Every step and observable runs in the library (FP64).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import configs, inputs, le, series


def _pick(table, sets):
    names = list(table)
    if sets:
        names = [n for n in sets.split(",") if n]
        bad = [n for n in names if n not in table]
        if bad:
            raise SystemExit(f"unknown sets {bad}; choose from {list(table)}")
    return [(list(table).index(n), n) for n in names]


def dv_sheared(strain: float, samples: int, refine: int = 1, sets: str = ""):
    for k, name in _pick(configs.DV_SHEARED, sets):
        p = configs.dv_sheared(name, refine)
        steps = int(round(strain / (p["gdot"] * p["dt"])))
        every = max(1, steps // samples)
        phi0 = inputs.noise_phi0(p["ny"], p["nx"], 500 + k, amp=configs.DV_AMP)
        def progress(done, o, name=name, every=every):
            if (done // every) % 10 == 0:
                print(f"{name}: strain {o['strain']:.1f}", file=sys.stderr, flush=True)

        try:
            r = series.run_series(p, phi0, steps, every, on_sample=progress)
        except (le.LeError, FloatingPointError) as ex:
            print(json.dumps({"set": name, "stopped": str(ex)}), flush=True)
            continue
        print(json.dumps({"set": name, "grid": [p["nx"], p["ny"]], "dt": p["dt"],
                          "steps": steps, "wall_s": r["wall_s"],
                          "site_updates_per_s": r["site_updates_per_s"],
                          "strain": r["strain"].tolist(), "L_par": r["L_par"].tolist(),
                          "L_perp": r["L_perp"].tolist()}), flush=True)


def _to_length(p, phi0, L_stop=0.025, chunk=250, max_chunks=1600):
    t, L = [], []
    with le.Context(p, phi0) as c:
        for _ in range(max_chunks):
            c.step(chunk)
            o, _ = c.observables(sk=False)
            t.append(o["t"])
            L.append(o["Ls"])
            if o["Ls"] >= L_stop:
                break
    return np.asarray(t), np.asarray(L)


def zero_shear(seeds: int, refine: int = 1, sets: str = ""):
    table = {**{n: configs.dv_unsheared(n, refine) for n in configs.DV_UNSHEARED},
             **{n: configs.r_unsheared(n, refine) for n in configs.R_UNSHEARED}}
    summary = {}
    for k, name in _pick(table, sets):
        p = table[name]
        ex = []
        for seed in range(seeds):
            phi0 = inputs.noise_phi0(p["ny"], p["nx"], 3000 + 100 * k + seed, amp=configs.DV_AMP)
            try:
                t, L = _to_length(p, phi0)
                e, ti, n = series.fit_power(t, L)
            except (le.LeError, ValueError) as err:
                print(json.dumps({"set": name, "seed": seed, "stopped": str(err)}), flush=True)
                continue
            ex.append(e)
            print(json.dumps({"set": name, "seed": seed, "t_end": float(t[-1]),
                              "exponent": e, "t_int": ti, "samples": n}), flush=True)
        if ex:
            summary[name] = {"mean": float(np.mean(ex)), "sd": float(np.std(ex)), "runs": len(ex)}
    print(json.dumps({"summary": summary}), flush=True)


def steady_states(strain: float, lb_sets: bool = False, refine: int = 1, sets: str = ""):
    rows = []
    table = configs.R_SHEARED_LB if lb_sets else configs.R_SHEARED
    for k, name in _pick(table, sets):
        p = configs.r_sheared(name, refine)
        steps = int(round(strain / (p["gdot"] * p["dt"])))
        phi0 = inputs.noise_phi0(p["ny"], p["nx"], (900 if lb_sets else 800) + k,
                                 amp=configs.DV_AMP)
        every = max(1, steps // 300)

        def progress(done, o, name=name, every=every):
            if (done // every) % 30 == 0:
                print(f"{name}: strain {o['strain']:.1f}", file=sys.stderr, flush=True)

        try:
            r = series.run_series(p, phi0, steps, every, on_sample=progress)
        except (le.LeError, FloatingPointError) as ex:
            print(json.dumps({"set": name, "stopped": str(ex)}), flush=True)
            continue
        avg = series.steady_average(r, 100.0)
        L_VI, t_VI = series.visco_inertial_scales(p)
        row = {"set": name, "grid": [p["nx"], p["ny"]], "dt": p["dt"], "steps": steps,
               "wall_s": r["wall_s"], "gdot_t_VI": p["gdot"] * t_VI, "L_VI": L_VI, **avg}
        rows.append(row)
        print(json.dumps(row), flush=True)
    if lb_sets or len(rows) < 3:
        return
    x = [r["gdot_t_VI"] for r in rows]
    ep = series.power_fit(x, [r["L_par"] / r["L_VI"] for r in rows])
    eq = series.power_fit(x, [r["L_perp"] / r["L_VI"] for r in rows])
    print(json.dumps({"summary": {"L_par_exponent": ep, "L_perp_exponent": eq}}), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("dv-sheared")
    a.add_argument("--strain", type=float, default=80.0)
    a.add_argument("--samples", type=int, default=100)
    b = sub.add_parser("zero-shear")
    b.add_argument("--seeds", type=int, default=4)
    for x in (a, b):
        x.add_argument("--refine", type=int, default=1, choices=(1, 2),
                       help="2: half the mesh interval of Table I at the same l")
        x.add_argument("--sets", default="", help="comma-separated subset of the sets")
    c = sub.add_parser("steady-states")
    c.add_argument("--strain", type=float, default=150.0)
    c.add_argument("--lb-sets", action="store_true",
                   help="the sets R028s, R022s, R029s instead of the scaling-plot sets")
    c.add_argument("--refine", type=int, default=1, choices=(1, 2),
                   help="2: half the mesh interval of Table I at the same l")
    c.add_argument("--sets", default="", help="comma-separated subset of the sets")
    args = ap.parse_args(argv)
    t0 = time.time()
    if args.cmd == "dv-sheared":
        dv_sheared(args.strain, args.samples, args.refine, args.sets)
    elif args.cmd == "zero-shear":
        zero_shear(args.seeds, args.refine, args.sets)
    else:
        steady_states(args.strain, args.lb_sets, args.refine, args.sets)
    print(json.dumps({"wall_s": time.time() - t0}), file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
