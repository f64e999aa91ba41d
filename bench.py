"""Throughput of the sheared model-H time step on one MI355X.

Headline workload (the largest single-GPU configuration): 4096 x 4096 grid,
spacing 1, A = B = kappa = M = eta = 1, rho = 1 (inertial), gdot = 0.001,
dt = 0.005, phi0 uniform in [-0.05, 0.05] (seed 0), omega0 = 0, FP64; the
observables (mean phi, L(t), S(k), excess stress) every 500 steps and at the
end of the timed region, inside it.  A step is one pass of every stage of the
split step.  Before the clock starts, every step-call length that the timed
region uses has been run once, so every captured graph piece exists.  Prints
one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, vendor figure
METRIC = "site-updates/s/GPU (plain FP64 vs FP32, batched, learned corrector) at stated L(t) error"


def stage_bytes(params, precision):
    """Algorithmic HBM bytes per launch of each stage (compulsory reads + writes)."""
    w = 8 if precision == "fp64" else 4
    nx, ny = params["nx"], params["ny"]
    real = nx * ny * w
    spec = ny * (nx // 2 + 1) * 2 * w
    if params["rho"] > 0:
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


def step_bytes(params, precision):
    return sum(stage_bytes(params, precision).values())


def four_pass_bytes(params, precision):
    """The minimum of a four-pass schedule: 16 field passes inertial, 12 Stokes."""
    w = 8 if precision == "fp64" else 4
    return (16 if params["rho"] > 0 else 12) * w * params["nx"] * params["ny"]


def host_transfer(ctx, sites, steps, gpu_ms):
    """The boundary's host hand-over at the headline size: one le_get_state
    (phi, omega, psi to host FP64 arrays) and one le_set_state back, timed on
    the wall clock; the PCIe-inclusive rate charges both to the timed steps.
    Not the headline value (that starts with the state resident in HBM)."""
    t0 = time.perf_counter()
    st = ctx.get_state()
    t1 = time.perf_counter()
    ctx.set_state(st["phi"], st["omega"], st["psi"], st["step"], st["wraps"])
    t2 = time.perf_counter()
    ctx.close()
    total = gpu_ms * 1e-3 + (t1 - t0) + (t2 - t1)
    return dict(value=sites * steps / total, unit="site-updates/s", get_state_s=t1 - t0,
                set_state_s=t2 - t1, bytes_each_way=3 * 8 * sites,
                note="the timed steps plus one get_state and one set_state of the three "
                     "FP64 fields through host memory")


def call_plan(steps, obs_every):
    """Lengths of the step calls of the timed region (observables after each)."""
    plan, done = [], 0
    while done < steps:
        n = min(obs_every, steps - done)
        plan.append(n)
        done += n
    return plan


def run_variant(le, torch, params, precision, steps, warmup, obs_every, seed=0,
                stage_reps=20, keep=False):
    """Timed region: the call plan (graph-replayed steps, observables after
    each call), bracketed by HIP events on the library's stream.  Warm-up: W
    steps, then one call of every distinct length of the plan and one
    observables call, so no graph is captured inside the clock.  Then each
    stage timed on its own: stage_reps back-to-back launches of its autotuned
    kernels between HIP events on the same stream."""
    from paper_0710_5912_amd import inputs

    nx, ny = params["nx"], params["ny"]
    phi0 = inputs.noise_phi0(ny, nx, seed, amp=0.05)
    stream = torch.cuda.Stream()          # default priority; the library enqueues on it
    ctx = le.Context(params, phi0, precision=precision, stream=stream.cuda_stream)
    plan = call_plan(steps, obs_every)
    if warmup:
        ctx.step(warmup)
    for n in sorted(set(plan)):
        ctx.step(n)
    o0, _ = ctx.observables(sk=True)
    step0 = o0["step"]
    series = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for n in plan:
        ctx.step(n)
        o, sk = ctx.observables(sk=True)
        series.append((o["t"], o["Ls"], o["sigma_xy"], o["mean_phi"]))
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    times = {}
    if stage_reps:
        times = {s: ctx.time_stage(s, stage_reps) for s in le.STAGES}
    tuning = ctx.tuning()[0]
    out = dict(wall=wall, gpu_ms=gpu_ms, times=times, series=series, tuning=tuning,
               steps_before=step0, obs_calls=len(plan), last_obs=o, last_sk=sk)
    if keep:
        out["ctx"] = ctx
    else:
        ctx.close()
    return out


def _batch_nr_ef(v):
    return (2, 16) if v >= 256 else (2, 8) if v >= 192 else (4, 16)


def batch_fits(v, nx):
    """The batched form applies: at least one wavefront per transform group."""
    nr, ef = _batch_nr_ef(v)
    return nr * (nx // 2 // ef) >= 64


def batch_shape(v):
    nr, ef = _batch_nr_ef(v)
    return "%d rows per batch, %d values per thread" % (nr, ef)


def stage_kernels(tuning, inertial):
    """Kernels each stage launches under the autotuned variants."""
    a, nx = tuning["advect"], tuning["nx"]
    if a == 0:
        adv = "k_bracket"
    elif a == 1024:
        adv = "k_adv_upwind + k_row_r2c"
    elif a >= 128 and 512 <= nx <= 4096 and batch_fits(a, nx):
        adv = "k_adv_batch (%s)" % batch_shape(a)
    elif 64 <= a < 128 and 256 <= nx <= 1024:
        adv = "k_adv_strip_fft"
    else:
        adv = "k_adv_strip + k_row_r2c"
    sq = tuning["nx"] == tuning["ny"]
    m = tuning["mu_source"]
    if m == 0 or not sq:
        mu = "k_mu + k_bracket"
    elif m >= 128 and 512 <= nx <= 4096 and batch_fits(m, nx):
        mu = "k_mug_batch (%s)" % batch_shape(m)
    elif 64 <= m < 128 and 256 <= nx <= 2048:
        mu = "k_mug_strip_fft"
    else:
        mu = "k_mug_strip + k_row_r2c"
    return {"row_inv_flow": "k_row_c2r", "advect": adv, "column_ch": "k_column<COL_CH>",
            "row_inv_phi": "k_row_c2r", "mu_source": mu,
            "column_flow": "k_column<COL_FLOW>" if inertial else "k_column<COL_STOKES>"}


def roofline_rows(params, precision, times):
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

    path = os.path.join(ROOT, "profiles", f"modelh_{nx}x{nx}_{precision}_traffic.md")
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


def field_error(a, b):
    """Max-norm relative difference of the state fields (phi, psi) and of L_s."""
    import numpy as np

    sa, sb = a.get_state(), b.get_state()
    out = {}
    for k in ("phi", "psi"):
        out[k] = float(np.max(np.abs(sa[k] - sb[k])) / np.max(np.abs(sb[k])))
    oa, ka = a.observables(sk=True)
    ob, kb = b.observables(sk=True)
    out["Ls"] = abs(oa["Ls"] - ob["Ls"]) / ob["Ls"]
    good = kb > 1e-3 * kb.max()
    out["Sk"] = float(np.max(np.abs(ka[good] - kb[good]) / kb[good]))
    return out


def precision_error(le, torch, params, steps, seed=0):
    """FP32 bulk against FP64 after `steps` steps from the same phi0 (the FP64
    GPU path equals the FP64 oracle to 1e-10 in the tests, so this is the FP32
    error against the oracle to that accuracy)."""
    from paper_0710_5912_amd import inputs

    phi0 = inputs.noise_phi0(params["ny"], params["nx"], seed, amp=0.05)
    a = le.Context(params, phi0, precision="fp32")
    b = le.Context(params, phi0, precision="fp64")
    a.step(steps)
    b.step(steps)
    err = field_error(a, b)
    a.close()
    b.close()
    err["steps"] = steps
    return err


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
    """Batched rate, the same runs one after another through the single-run
    path (each warmed up with the timed call length first), and the FP32
    batch's error against single FP64 runs for a sample of runs."""
    import numpy as np

    params, phis = batch_workload()
    sites = sum(p["nx"] * p["ny"] for p in params)
    stream = torch.cuda.Stream()
    b = le.Batch(params, phis, precisions=["fp32"] * len(params), stream=stream.cuda_stream)
    b.step(warmup)
    b.step(steps)       # every graph piece of the timed call captured
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    batched = sites * steps / (e0.elapsed_time(e1) * 1e-3)
    done = warmup + 2 * steps
    sample = (0, 33, 66, 95)
    errs = []
    for r in sample:
        ref = le.Context(params[r], phis[r], precision="fp64")
        ref.step(done)
        sr, sb = ref.get_state(), b.get_state(r)
        errs.append(float(np.max(np.abs(sb["phi"] - sr["phi"])) / np.max(np.abs(sr["phi"]))))
        ref.close()
    b.close()
    total_ms = 0.0
    for p, phi0 in zip(params, phis):
        c = le.Context(p, phi0, precision="fp32", stream=stream.cuda_stream)
        c.step(seq_steps)       # capture the call's graph pieces
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
                error=dict(sample_runs=list(sample), steps=done,
                           phi_rel_err_vs_fp64_single_runs=errs,
                           note="each run is also bit-identical to its FP32 single run (tests)"))


def corrector_ensemble(corrector, cp, cs, seeds=tuple(range(90, 98)),
                       gdots=(0.003, 0.01, 0.03), t_end=100.0):
    """The corrector on held-out seeds at three shear rates (t = 20 .. t_end):
    mean errors of L(t) and S(k) of the corrected and the plain coarse run
    against the fine run (L) and its restriction (S(k)), per shear rate, and
    the fine-equivalent gain."""
    import numpy as np

    res = {}
    for g in gdots:
        evs = [corrector.evaluate(cp, cs, gdot=g, seed=s, t_end=t_end, log=lambda m: None)
               for s in seeds]
        pick = lambda k: [e[k] for e in evs]  # noqa: E731
        res[f"gdot_{g:g}"] = dict(
            L_err_mean=float(np.mean(pick("err_mean_corrected"))),
            L_err_mean_plain_coarse=float(np.mean(pick("err_mean_coarse"))),
            L_err_of_ensemble_mean=float(np.mean(np.abs(
                np.mean([e["corrected"] for e in evs], axis=0)
                - np.mean([e["fine"] for e in evs], axis=0))
                / np.mean([e["fine"] for e in evs], axis=0))),
            Sk_err_mean=float(np.mean(pick("Sk_err_mean_corrected"))),
            Sk_err_mean_plain_coarse=float(np.mean(pick("Sk_err_mean_coarse"))),
            Sk_low_err_mean=float(np.mean(pick("Sk_low_err_mean_corrected"))),
            Sk_low_err_mean_plain_coarse=float(np.mean(pick("Sk_low_err_mean_coarse"))),
            Sk_high_err_mean=float(np.mean(pick("Sk_high_err_mean_corrected"))),
            Sk_high_err_mean_plain_coarse=float(np.mean(pick("Sk_high_err_mean_coarse"))),
            gain=float(np.mean(pick("gain"))))
    return dict(seeds=list(seeds), t=[corrector.T_START, t_end], per_gdot=res,
                note="held-out seeds; L(t) errors against the plain 1024^2 FP64 run, S(k) "
                     "errors against its restriction to the coarse grid (shells up to half "
                     "the coarse Nyquist; low: 1 .. 32, the domain band; high: 32 .. 128, "
                     "the interface band), relative, averaged over the samples every 5 time "
                     "units; L_err_of_ensemble_mean: the 8-seed mean L(t) against the fine "
                     "8-seed mean")


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(params):
    """The FP64 oracle, untuned, on one step of the headline workload (a
    bounded sample: one 4096^2 oracle step is ~10-15 s of CPU work), then the
    same step with its 2D FFTs taken by scipy.fft over all host threads."""
    import numpy as np
    import scipy.fft as sf

    from oracle import model_h as mh
    from paper_0710_5912_amd import inputs

    model, nproc = cpu_info()
    p = mh.Params(**params)
    st = mh.initial_state(p, inputs.noise_phi0(p.ny, p.nx, 0, amp=0.05))
    t0 = time.perf_counter()
    st = mh.step(p, st)
    dt1 = time.perf_counter() - t0
    fft2, ifft2 = mh.fft2, mh.ifft2_real
    try:
        mh.fft2 = lambda a: sf.fft2(a, workers=nproc)
        mh.ifft2_real = lambda A: np.real(sf.ifft2(A, workers=nproc))
        t0 = time.perf_counter()
        st = mh.step(p, st)
        dtn = time.perf_counter() - t0
    finally:
        mh.fft2, mh.ifft2_real = fft2, ifft2
    assert np.isfinite(st.phi).all()
    sites = p.nx * p.ny
    return dict(value=sites / dt1, unit="site-updates/s", cores=1, kind="oracle",
                sample=f"1 step of the {p.nx}x{p.ny} FP64 inertial headline workload "
                       f"({dt1:.1f} s; NumPy FFTs and ufuncs, one thread)",
                cpu_model=model, nproc=nproc,
                threaded=dict(value=sites / dtn, cores=nproc,
                              sample=f"the next step with scipy.fft workers={nproc} for the "
                                     f"2D FFTs ({dtn:.1f} s); stencils single-threaded"))


def variant_entry(params, precision, rv, steps, sites):
    d, rw = roofline_rows(params, precision, rv["times"])
    ms = rv["gpu_ms"] / steps
    return dict(value=sites * steps / (rv["gpu_ms"] * 1e-3), ms_per_step=ms,
                dominant=d, dominant_frac=rw[d]["gbs"] / HBM_PEAK_GBS,
                step_frac=step_bytes(params, precision) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                step_frac_four_pass=four_pass_bytes(params, precision) / (ms * 1e-3) / 1e9
                / HBM_PEAK_GBS,
                tuning=rv["tuning"], obs_calls=rv["obs_calls"],
                stages={k: {"avg_us": round(v["avg_us"], 1), "GBs": round(v["gbs"], 1)}
                        for k, v in rw.items()})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--obs-every", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32"),
                    help="headline precision (the configuration's default: fp64)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="short pass for hardware counters: a 512 MiB device copy "
                         "(calibration of FETCH_SIZE/WRITE_SIZE) then directly launched "
                         "steps of the headline workload; prints no JSON")
    ap.add_argument("--profile-size", type=int, default=4096)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the time step of one grid is not sharded across GPUs here)", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    from paper_0710_5912_amd import configs, inputs, le

    params = configs.LARGE_4096["params"]
    prec = args.precision
    if args.profile_pass:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        n = args.profile_size
        pp = configs.model_h(n, n, gdot=params["gdot"] if n == 4096 else 0.01, rho=1.0)
        ctx = le.Context(pp, inputs.noise_phi0(n, n, 0), precision=prec)
        ctx.profile(True)      # direct launches: one dispatch per stage and step
        ctx.step(10 if n >= 4096 else 50)
        print(json.dumps({"profile_pass": ctx.stage_times(), "tuning": ctx.tuning()}))
        ctx.close()
        return
    nx, ny = params["nx"], params["ny"]
    sites = nx * ny
    print(f"bench: {nx}x{ny} {prec} inertial, {args.warmup} warmup + {args.steps} timed steps",
          file=sys.stderr, flush=True)
    r = run_variant(le, torch, params, prec, args.steps, args.warmup, args.obs_every,
                    keep=True)
    pcie = host_transfer(r.pop("ctx"), sites, args.steps, r["gpu_ms"])
    copy_gbs = copy_bandwidth(torch)
    value = sites * args.steps / (r["gpu_ms"] * 1e-3)
    dom, rows = roofline_rows(params, prec, r["times"])
    ms_step = r["gpu_ms"] / args.steps
    o = r["last_obs"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"sheared model H, {nx}x{ny}, inertial rho=1, eta=1, "
                               f"gdot=0.001, dt=0.005, A=B=kappa=M=1, dx=1, phi0 "
                               f"U(-0.05,0.05) seed 0, omega0=0, plain {prec.upper()} step, "
                               f"observables (L(t), S(k), stress) every {args.obs_every} "
                               f"steps and at the end, inside the timed region",
                   "grid": [nx, ny], "precision": prec, "rho": 1.0, "gdot": 0.001,
                   "obs_every": args.obs_every, "obs_calls": r["obs_calls"],
                   "warmup_note": "W steps, then one call of each timed call length and "
                                  "one observables call before the clock starts"},
        "roofline": {"bound": "hbm", "stage": dom,
                     "kernels": stage_kernels(r["tuning"], True)[dom],
                     "timing": f"HIP events around back-to-back launches of the stage's "
                               f"autotuned kernels on the library's stream, after the timed "
                               f"region",
                     "achieved": rows[dom]["gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": rows[dom]["gbs"] / HBM_PEAK_GBS,
                     "traffic": traffic_of(dom, prec, nx, r["tuning"]),
                     "bytes_per_launch": rows[dom]["bytes"],
                     "avg_launch_us": rows[dom]["avg_us"],
                     "copy_gbs": copy_gbs,
                     "copy_note": "512 MiB device-to-device tensor copy (runtime copy kernel), "
                                  "bytes read + written, timed after the bench",
                     "frac_of_copy": rows[dom]["gbs"] / copy_gbs},
        "stages": {k: {"avg_us": round(v["avg_us"], 2), "GBs": round(v["gbs"], 1)}
                   for k, v in rows.items()},
        "step_roofline": {"bytes_per_step": step_bytes(params, prec),
                          "bytes_per_step_four_pass_minimum": four_pass_bytes(params, prec),
                          "frac": step_bytes(params, prec) / (ms_step * 1e-3) / 1e9
                          / HBM_PEAK_GBS,
                          "frac_four_pass_minimum": four_pass_bytes(params, prec)
                          / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "last_observables": {k: o[k] for k in ("step", "t", "mean_phi", "Ls", "L_par",
                                                "L_perp", "sigma_xy", "sigma_xy_re")},
        "pcie_inclusive": pcie,
        "tuning": r["tuning"],
        "wall_s": r["wall"],
        "hip_note": le.lib().le_last_error().decode(),
        "error": "FP64 path within 1e-10 (max norm, relative) of the FP64 oracle after 100 "
                 "steps in the parity tests, and at sampled points of this workload",
    }
    if not args.no_variants:
        var = {}
        print("bench: variant fp32 4096", file=sys.stderr, flush=True)
        p = configs.LARGE_4096["params"]
        rv = run_variant(le, torch, p, "fp32", 1000, 100, 500)
        var["fp32_4096_inertial"] = variant_entry(p, "fp32", rv, 1000, sites)
        var["fp32_4096_inertial"]["error_vs_fp64"] = precision_error(le, torch, p, 200)
        for name, prec_v, rho in (("fp64_1024_inertial", "fp64", 1.0),
                                  ("fp32_1024_inertial", "fp32", 1.0),
                                  ("fp64_1024_stokes", "fp64", 0.0),
                                  ("fp32_1024_stokes", "fp32", 0.0)):
            p = configs.single_1024(rho=rho, gdot=0.01)["params"]
            print(f"bench: variant {name}", file=sys.stderr, flush=True)
            rv = run_variant(le, torch, p, prec_v, 2000, 100, 100, stage_reps=100)
            var[name] = variant_entry(p, prec_v, rv, 2000, 1024 * 1024)
            if prec_v == "fp32":
                var[name]["error_vs_fp64"] = precision_error(le, torch, p, 2000)
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
            Sk_err_mean=ev["Sk_err_mean_corrected"],
            Sk_err_mean_plain_coarse=ev["Sk_err_mean_coarse"],
            Sk_low_err_mean=ev["Sk_low_err_mean_corrected"],
            Sk_low_err_mean_plain_coarse=ev["Sk_low_err_mean_coarse"],
            Sk_high_err_mean=ev["Sk_high_err_mean_corrected"],
            Sk_high_err_mean_plain_coarse=ev["Sk_high_err_mean_coarse"],
            audited_value=ev["audited_fine_equiv_rate"], audit=ev["audit"],
            audited_equals_corrected=ev["audited_equals_corrected"],
            note=f"fine-equivalent site-updates/s of 256^2 corrected steps at 4 dt against "
                 f"the 1024^2 FP64 plain run, t = {corrector.T_START:g}..{corrector.T_END:g}, "
                 f"gdot = 0.01, held-out seed; errors of L(t) against the fine run and "
                 f"against the fine field restricted to the coarse grid; audited: the "
                 f"corrected run with a 20-step corrected-vs-plain audit every 500 steps "
                 f"(L_s tolerance 2%)")
        evp = corrector.evaluate(cp, cs, gdot=0.01, seed=99, log=lambda m: None, projection=1)
        var["corrector_256_from_1024"]["projection_1"] = dict(
            value=evp["corrected_fine_equiv_rate"], gain=evp["gain"],
            L_err_mean=evp["err_mean_corrected"], L_err_max=evp["err_max_corrected"],
            Sk_low_err_mean=evp["Sk_low_err_mean_corrected"],
            Sk_high_err_mean=evp["Sk_high_err_mean_corrected"],
            note="the same run with the phi residual's interpolated 16 x 16 tile means "
                 "subtracted instead of its mean")
        print("bench: variant corrector at 4096^2 / 1024^2", file=sys.stderr, flush=True)
        ev5 = corrector.evaluate(cp, cs, gdot=0.001, seed=99, t_end=100.0, n=4096,
                                 log=lambda m: None)
        var["corrector_1024_from_4096_extrapolation"] = dict(
            value=ev5["corrected_fine_equiv_rate"], plain_fine_value=ev5["fine_rate"],
            gain=ev5["gain"], L_err_mean=ev5["err_mean_corrected"],
            L_err_mean_plain_coarse=ev5["err_mean_coarse"],
            Sk_low_err_mean=ev5["Sk_low_err_mean_corrected"],
            Sk_low_err_mean_plain_coarse=ev5["Sk_low_err_mean_coarse"],
            Sk_high_err_mean=ev5["Sk_high_err_mean_corrected"],
            Sk_high_err_mean_plain_coarse=ev5["Sk_high_err_mean_coarse"],
            note="the network trained on 1024^2 -> 256^2 data (gdot 0.003 .. 0.03) applied to "
                 "a 4096^2 FP64 run restricted to 1024^2 (4 dt coarse steps) at gdot = 0.001, "
                 "t = 20 .. 100, seed 99: an extrapolation in system size and shear rate; "
                 "fine-equivalent rate = 4096^2 sites x fine steps / corrected wall time")
        print("bench: variant corrector ensemble", file=sys.stderr, flush=True)
        var["corrector_ensemble_8_seeds"] = corrector_ensemble(corrector, cp, cs)
        out["variants"] = var
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(params)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
