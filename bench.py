"""Throughput of the sheared model-H time step on one MI355X.

Workload (the single-run configuration): 1024 x 1024 grid, spacing 1,
A = B = kappa = M = eta = 1, rho = 1, gdot = 0.01, dt = 0.005, phi0 uniform in
[-0.05, 0.05] (seed 0), omega0 = 0; observables (L(t), S(k), stress) every 100
steps inside the timed region.  A step is one pass of every stage of the split
step.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, vendor figure


def stage_bytes(params, precision):
    """Algorithmic HBM bytes per launch of each stage (compulsory reads + writes)."""
    w = 8 if precision == "fp64" else 4
    nx, ny = params["nx"], params["ny"]
    real = nx * ny * w
    spec = ny * (nx // 2 + 1) * 2 * w
    inertial = params["rho"] > 0
    if inertial:
        return {
            "row_inv_flow": 2 * spec + 2 * real,
            "advect": 3 * real + 3 * spec,
            "column_ch": 3 * spec,
            "row_inv_phi": spec + real,
            "mu_source": real + spec,
            "column_flow": 4 * spec,
        }
    return {
        "row_inv_flow": spec + real,
        "advect": 2 * real + 2 * spec,
        "column_ch": 3 * spec,
        "row_inv_phi": spec + real,
        "mu_source": real + spec,
        "column_flow": 2 * spec,
    }


def run_variant(le, torch, params, precision, steps, warmup, obs_every, seed=0,
                stage_reps=200):
    """Timed region (graph-replayed steps, observables every obs_every steps),
    then each stage timed on its own: stage_reps back-to-back launches of its
    (autotuned) kernels between HIP events on the same stream."""
    from paper_0710_5912_amd import inputs

    nx, ny = params["nx"], params["ny"]
    phi0 = inputs.noise_phi0(ny, nx, seed, amp=0.05)
    stream = torch.cuda.Stream()          # default priority; the library enqueues on it
    ctx = le.Context(params, phi0, precision=precision, stream=stream.cuda_stream)
    ctx.step(warmup)
    series = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    done = 0
    while done < steps:
        n = min(obs_every, steps - done)
        ctx.step(n)
        done += n
        if done % obs_every == 0:
            o, _ = ctx.observables(sk=True)
            series.append((o["t"], o["Ls"], o["sigma_xy"], o["mean_phi"]))
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    times = {}
    if stage_reps:
        times = {s: ctx.time_stage(s, stage_reps) for s in le.STAGES}
    tuning = ctx.tuning()[0]
    ctx.close()
    return dict(wall=wall, gpu_ms=gpu_ms, times=times, series=series, tuning=tuning)


def step_bytes(params, precision):
    return sum(stage_bytes(params, precision).values())


def stage_kernels(tuning, inertial):
    """Kernels each stage launches under the autotuned variants."""
    a = tuning["advect"]
    fused_strip = a >= 64 and 256 <= tuning["nx"] <= 1024
    adv = ("k_bracket" if a == 0 else
           ("k_adv_strip_fft" if fused_strip else "k_adv_strip + k_row_r2c"))
    sq = tuning["nx"] == tuning["ny"]
    m = tuning["mu_source"]
    mu = ("k_mu + k_bracket" if m == 0 or not sq else
          ("k_mug_strip_fft" if m >= 64 and 256 <= tuning["nx"] <= 2048
           else "k_mug_strip + k_row_r2c"))
    return {"row_inv_flow": "k_row_c2r", "advect": adv, "column_ch": "k_column<COL_CH>",
            "row_inv_phi": "k_row_c2r", "mu_source": mu,
            "column_flow": "k_column<COL_FLOW>" if inertial else "k_column<COL_STOKES>"}


def batch_workload():
    """96 runs: 32 each of 128^2, 256^2, 512^2; gdot log-uniform in [1e-3, 1e-1]
    (seed 1000); rho alternating 0 / 1; phi0 seed 2000 + r; FP32 bulk."""
    from paper_0710_5912_amd import configs, inputs

    gd = inputs.batch_draws(96, seed=1000)
    params, phis = [], []
    for r in range(96):
        n = (128, 256, 512)[r // 32]
        params.append(configs.model_h(n, n, gdot=float(gd[r]), rho=float(r % 2)))
        phis.append(inputs.noise_phi0(n, n, 2000 + r, amp=0.05))
    return params, phis


def run_batch(le, torch, steps, warmup, seq_steps):
    params, phis = batch_workload()
    sites = sum(p["nx"] * p["ny"] for p in params)
    stream = torch.cuda.Stream()
    b = le.Batch(params, phis, precisions=["fp32"] * len(params), stream=stream.cuda_stream)
    b.step(warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    batched = sites * steps / (e0.elapsed_time(e1) * 1e-3)
    b.close()
    # the same runs one after another through the single-run path
    total_ms = 0.0
    for p, phi0 in zip(params, phis):
        c = le.Context(p, phi0, precision="fp32", stream=stream.cuda_stream)
        c.step(10)
        torch.cuda.synchronize()
        e0.record(stream)
        c.step(seq_steps)
        e1.record(stream)
        torch.cuda.synchronize()
        total_ms += e0.elapsed_time(e1)
        c.close()
    sequential = sites * seq_steps / (total_ms * 1e-3)
    return dict(value=batched, sequential_value=sequential, gain=batched / sequential,
                runs=len(params), sites=sites, steps=steps,
                error="each run bit-identical to its single-run result (tests)")


def roofline_of(params, precision, times):
    """Per stage: average launch us, algorithmic bytes and GB/s; the dominant stage."""
    b = stage_bytes(params, precision)
    rows = {k: dict(avg_us=us, bytes=b[k], gbs=b[k] / (us * 1e-6) / 1e9)
            for k, us in times.items()}
    if not rows:
        return None, {}
    dom = max(rows, key=lambda k: rows[k]["avg_us"])
    return dom, rows


def traffic_of(stage, precision, nx, tuning):
    """HBM bytes per launch of `stage` from the committed rocprofv3 counter record
    (one entry per variant of each stage), or None when there is none for this
    workload or variant, or the kernel sources changed since."""
    import glob
    import hashlib

    if precision != "fp64" or nx != 1024:
        return None
    path = os.path.join(ROOT, "profiles", "modelh_1024x1024_fp64_traffic.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_0710_5912_amd", "csrc", "*"))):
        h.update(open(p, "rb").read())
    if rec is None or rec["source_hash"] != h.hexdigest()[:16] or stage not in rec["stages"]:
        return None
    key = rec.get("variant_key", {}).get(stage)
    k = rec["stages"][stage].get(str(tuning[key])) if key in tuning else None
    if k is None:
        return None
    return (k["fetch_kib"] * rec["fetch_factor"] + k["write_kib"] * rec["write_factor"]) * 1024.0


def copy_bandwidth(torch, mib=512, reps=20):
    """Measured device-to-device copy bandwidth (GB/s, bytes read + written):
    the second denominator of the roofline fractions."""
    src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * src.numel() * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def cpu_baseline(params, budget_s=15.0):
    """The FP64 oracle, untuned, on a bounded number of steps of the same workload."""
    import numpy as np

    from oracle import model_h as mh
    from paper_0710_5912_amd import inputs

    p = mh.Params(**params)
    phi0 = inputs.noise_phi0(p.ny, p.nx, 0, amp=0.05)
    st = mh.initial_state(p, phi0)
    st = mh.step(p, st)           # first step outside the clock (allocations)
    t0 = time.perf_counter()
    n = 0
    while True:
        st = mh.step(p, st)
        n += 1
        if time.perf_counter() - t0 >= budget_s and n >= 3:
            break
    dt = time.perf_counter() - t0
    assert np.isfinite(st.phi).all()
    return dict(value=p.nx * p.ny * n / dt, unit="site-updates/s", cores=1, kind="oracle",
                sample=f"{n} steps of the {p.nx}x{p.ny} inertial workload after 1 untimed "
                       f"step ({dt:.1f} s); NumPy FFT and ufuncs, single thread")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--obs-every", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--profile-size", type=int, default=1024)
    ap.add_argument("--profile-precision", default="fp64", choices=("fp64", "fp32"))
    ap.add_argument("--profile-pass", action="store_true",
                    help="short pass for hardware counters: a 512 MiB device copy "
                         "(calibration of FETCH_SIZE/WRITE_SIZE) then 50 directly launched "
                         "steps of the 1024^2 FP64 workload; prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the time step of one grid is not sharded across GPUs here)", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    from paper_0710_5912_amd import configs, le

    params = configs.single_1024(rho=1.0, gdot=0.01)["params"]
    if args.profile_pass:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        from paper_0710_5912_amd import inputs
        n = args.profile_size
        pp = configs.model_h(n, n, gdot=0.01, rho=1.0)
        ctx = le.Context(pp, inputs.noise_phi0(n, n, 0), precision=args.profile_precision)
        ctx.profile(True)      # direct launches: one dispatch per stage and step
        ctx.step(50 if n <= 1024 else 10)
        print(json.dumps({"profile_pass": ctx.stage_times(), "tuning": ctx.tuning()}))
        ctx.close()
        return
    print(f"bench: 1024x1024 fp64 inertial, {args.warmup} warmup + {args.steps} timed steps",
          file=sys.stderr, flush=True)
    r = run_variant(le, torch, params, "fp64", args.steps, args.warmup, args.obs_every)
    sites = params["nx"] * params["ny"]
    copy_gbs = copy_bandwidth(torch)
    sec = r["gpu_ms"] * 1e-3
    value = sites * args.steps / sec
    dom, rows = roofline_of(params, "fp64", r["times"])
    out = {
        "metric": "site-updates/s/GPU (plain FP64 vs FP32, batched, learned corrector) at stated L(t) error",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["gpu_ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sheared model H, 1024x1024, inertial rho=1, eta=1, gdot=0.01, "
                               "dt=0.005, A=B=kappa=M=1, dx=1, phi0 U(-0.05,0.05) seed 0, "
                               "plain FP64 step, observables every 100 steps",
                   "grid": [1024, 1024], "precision": "fp64", "rho": 1.0, "gdot": 0.01,
                   "obs_every": args.obs_every},
        "roofline": {"bound": "hbm", "stage": dom,
                     "kernels": stage_kernels(r["tuning"], True)[dom],
                     "timing": "HIP events around 200 back-to-back launches of the stage's "
                               "kernels after the timed region, on the library's stream",
                     "achieved": rows[dom]["gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": rows[dom]["gbs"] / HBM_PEAK_GBS,
                     "traffic": traffic_of(dom, "fp64", 1024, r["tuning"]),
                     "bytes_per_launch": rows[dom]["bytes"],
                     "avg_launch_us": rows[dom]["avg_us"],
                     "copy_gbs": copy_gbs,
                     "copy_note": "512 MiB device-to-device tensor copy (runtime copy kernel), "
                                  "bytes read + written, timed after the bench",
                     "frac_of_copy": rows[dom]["gbs"] / copy_gbs},
        "stages": {k: {"avg_us": round(v["avg_us"], 2), "GBs": round(v["gbs"], 1)}
                   for k, v in rows.items()},
        "step_roofline": {"bytes_per_step": step_bytes(params, "fp64"),
                          "bytes_per_step_four_pass_minimum": 128 * sites,
                          "frac": step_bytes(params, "fp64") / (r["gpu_ms"] / args.steps * 1e-3)
                          / 1e9 / HBM_PEAK_GBS,
                          "frac_four_pass_minimum": 128 * sites / (r["gpu_ms"] / args.steps * 1e-3)
                          / 1e9 / HBM_PEAK_GBS},
        "tuning": r["tuning"],
        "wall_s": r["wall"],
        "hip_note": le.lib().le_last_error().decode(),
        "parity": "FP64 path within 1e-10 of the FP64 oracle after 100 steps (tests)",
    }
    if not args.no_variants:
        var = {}
        for name, prec, rho, n in (("fp32_inertial", "fp32", 1.0, 2000),
                                   ("fp64_stokes", "fp64", 0.0, 2000),
                                   ("fp32_stokes", "fp32", 0.0, 2000)):
            p = configs.single_1024(rho=rho, gdot=0.01)["params"]
            print(f"bench: variant {name}", file=sys.stderr, flush=True)
            rv = run_variant(le, torch, p, prec, n, 100, args.obs_every)
            d, rw = roofline_of(p, prec, rv["times"])
            var[name] = dict(value=sites * n / (rv["gpu_ms"] * 1e-3),
                             ms_per_step=rv["gpu_ms"] / n,
                             dominant=d, dominant_frac=rw[d]["gbs"] / HBM_PEAK_GBS,
                             tuning=rv["tuning"])
        print("bench: variant batched_96", file=sys.stderr, flush=True)
        var["batched_96_fp32"] = run_batch(le, torch, 500, 50, 100)
        print("bench: variant corrector", file=sys.stderr, flush=True)
        from paper_0710_5912_amd import corrector
        cp, cs, meta = corrector.load()
        ev = corrector.evaluate(cp, cs, gdot=0.01, seed=99, log=lambda m: None,
                                audit=(500, 20, 0.02))
        var["corrector_256_from_1024"] = dict(
            value=ev["corrected_fine_equiv_rate"], plain_fine_value=ev["fine_rate"],
            gain=ev["gain"], L_err_mean=ev["err_mean_corrected"],
            L_err_max=ev["err_max_corrected"], L_err_mean_plain_coarse=ev["err_mean_coarse"],
            L_err_mean_vs_restricted=ev["err_mean_corrected_vs_restricted"],
            L_err_max_vs_restricted=ev["err_max_corrected_vs_restricted"],
            L_err_mean_plain_coarse_vs_restricted=ev["err_mean_coarse_vs_restricted"],
            L_restriction_bias=ev["err_mean_restriction"],
            audited_value=ev["audited_fine_equiv_rate"], audit=ev["audit"],
            audited_equals_corrected=ev["audited_equals_corrected"],
            note=f"fine-equivalent site-updates/s of 256^2 corrected steps at 4 dt against "
                 f"the 1024^2 FP64 plain run, t = {corrector.T_START:g}..{corrector.T_END:g}, "
                 f"gdot = 0.01, held-out seed; errors of L(t) against the fine run and "
                 f"against the fine field restricted to the coarse grid; audited: the "
                 f"corrected run with a 20-step corrected-vs-plain audit every 500 steps "
                 f"(L_s tolerance 2%)")
        # the inertialess sheared set DV4s of Table I in paper units (1024 x 512,
        # Stokes branch), 20000 steps with observables every 5000
        print("bench: variant dv4s", file=sys.stderr, flush=True)
        from paper_0710_5912_amd import inputs, series
        pdv = configs.dv_sheared("DV4s")
        rdv = series.run_series(pdv, inputs.noise_phi0(512, 1024, 500, amp=configs.DV_AMP),
                                20000, 5000)
        var["dv4s_1024x512_stokes_fp64"] = dict(
            value=rdv["site_updates_per_s"], steps=20000, strain=float(rdv["strain"][-1]),
            L_par=float(rdv["L_par"][-1]), L_perp=float(rdv["L_perp"][-1]),
            note="Table I set DV4s (eta = 1, gdot = 0.01, l = 0.00156, rho = 0, box 2 x 1), "
                 "wall time of stepping plus observables every 5000 steps")
        # the large single-GPU grid, FP64 and FP32 bulk
        for prec in ("fp64", "fp32"):
            p = configs.LARGE_4096["params"]
            print(f"bench: variant {prec}_4096", file=sys.stderr, flush=True)
            rv = run_variant(le, torch, p, prec, 200, 20, 100, stage_reps=20)
            d, rw = roofline_of(p, prec, rv["times"])
            ms = rv["gpu_ms"] / 200
            var[f"{prec}_4096_inertial"] = dict(
                value=4096 * 4096 * 200 / (rv["gpu_ms"] * 1e-3), ms_per_step=ms, dominant=d,
                dominant_frac=rw[d]["gbs"] / HBM_PEAK_GBS,
                step_frac=step_bytes(p, prec) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                tuning=rv["tuning"],
                stages={k: {"avg_us": round(v["avg_us"], 1), "GBs": round(v["gbs"], 1)}
                        for k, v in rw.items()})
        out["variants"] = var
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(params)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
