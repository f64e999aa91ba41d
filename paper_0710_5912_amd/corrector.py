"""Data generation, training and evaluation of the learned coarse-step corrector.

Orchestration only: every step, restriction, network pass and optimiser
update runs in the HIP library (paper_0710_5912_amd.le); torch holds the
training tensors in device memory.

Workload (the corrector configuration): fine runs on a 1024 x 1024 grid
(spacing 1, FP64, rho = eta = 1, dt = 0.005, A = B = 1, kappa = M = 8: the
paper's units with interface length l = 2 sqrt 2 grid spacings, so that the
interface spans most of a coarse cell) at shear rates in [0.003, 0.03] are
sampled at t = 20 .. 300; each sample is restricted by 4 x 4 block means to
the 256 x 256 coarse grid (spacing 4), advanced by one plain coarse step of
4 dt = 0.02, and paired with the restricted fine state 4 fine steps later.
The network learns the residual between the two; at inference it corrects
each coarse step.  (With kappa = 1 the interface is a third of a coarse
cell and no coarse model follows the fine L(t); with kappa = M = 16 the
explicit advection of this scheme loses stability near t ~ 100 at dt =
0.005.)

L(t) errors are reported against the fine run's L(t) and against L(t) of
the restricted fine field (the same field seen on the coarse grid: the
comparison the coarse solution can be expected to match).

    python -m paper_0710_5912_amd.corrector train --out weights.npz
    python -m paper_0710_5912_amd.corrector eval --weights weights.npz
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import configs, inputs, le

FINE_N = 1024
FACTOR = 4
DT = 0.005
KAPPA = 8.0    # kappa = M = l^2
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "corrector_c4.npz")


def fine_params(gdot, n=FINE_N):
    return configs.model_h(n, n, gdot=gdot, rho=1.0, dt=DT, kappa=KAPPA, M=KAPPA)


def coarse_params(gdot, n=FINE_N, factor=FACTOR):
    nc = n // factor
    return configs.model_h(nc, nc, gdot=gdot, rho=1.0, dt=DT * factor, lx=float(n),
                           ly=float(n), kappa=KAPPA, M=KAPPA)


def _wraps(params, n):
    c = params["lx"] / params["ly"]
    X = params["gdot"] * (float(n) * params["dt"])
    return math.floor((X + 0.5 * c) / c)


T_START, T_END = 20.0, 300.0


def generate_pairs(n_pairs=2000, gdots=(0.003, 0.005, 0.008, 0.012, 0.018, 0.03),
                   seeds=(11, 12, 13, 14, 15, 16), t_start=T_START, t_end=T_END, n=FINE_N,
                   factor=FACTOR, log=print):
    """(x, t) pairs: x = coarse-stepped restricted state, t = target residual."""
    per_run = -(-n_pairs // len(gdots))
    k0 = int(round(t_start / DT))
    k1 = int(round(t_end / DT))
    stride = max(factor, ((k1 - k0) // per_run) // factor * factor)
    xs, ts = [], []
    for gdot, seed in zip(gdots, seeds):
        fp = fine_params(gdot, n)
        cp = coarse_params(gdot, n, factor)
        nc = n // factor
        fine = le.Context(fp, inputs.noise_phi0(n, n, seed, amp=0.05))
        coarse = le.Context(cp, np.zeros((nc, nc)))
        fine.step(k0)
        step = k0
        got = 0
        t0 = time.time()
        while got < per_run and step + factor <= k1:
            phi_c, om_c = fine.restrict(factor)
            fine.step(factor)
            phi_n, om_n = fine.restrict(factor)
            if _wraps(fp, step) == _wraps(fp, step + factor):   # skip steps across a wrap
                coarse.set_fields(phi_c, om_c, step // factor)
                coarse.step(1)
                g = coarse.get_state()
                xs.append(np.stack([g["phi"], g["omega"]]).astype(np.float32))
                ts.append(np.stack([phi_n - g["phi"], om_n - g["omega"]]).astype(np.float32))
                got += 1
            fine.step(stride - factor)
            step += stride
        fine.close()
        coarse.close()
        log(f"corrector data: gdot={gdot} seed={seed} pairs={got} ({time.time() - t0:.1f} s)")
    return np.stack(xs[:n_pairs]), np.stack(ts[:n_pairs])


def scales_from(xs, ts):
    """Per-channel input and output scales: inputs and targets at unit RMS."""
    def rms(a):
        return float(np.sqrt(np.mean(a.astype(np.float64) ** 2))) or 1.0
    return np.array([1.0 / rms(xs[:, 0]), 1.0 / rms(xs[:, 1]), rms(ts[:, 0]), rms(ts[:, 1])],
                    dtype=np.float32)


def train(xs, ts, epochs=20, batch=16, lr=1e-3, seed=0, log=print):
    import torch

    nc = xs.shape[-1]
    scales = scales_from(xs, ts)
    net = le.Net(nc, nc)
    net.set_params(inputs.cnn_init_params(seed).astype(np.float32), scales)
    X = torch.tensor(xs, device="cuda")
    T = torch.tensor(ts, device="cuda")
    rng = np.random.default_rng(seed)
    n = xs.shape[0]
    history = []
    for ep in range(epochs):
        order = rng.permutation(n)
        tot = 0.0
        for b in range(0, n - batch + 1, batch):
            idx = torch.tensor(order[b:b + batch], device="cuda")
            loss, _ = net.grad(X[idx].contiguous(), T[idx].contiguous(), batch)
            net.adam(lr * (0.5 ** (ep // 8)))
            tot += loss
        mean = tot / (n // batch)
        history.append(mean)
        log(f"corrector train: epoch {ep} loss {mean:.4e} (relative {mean:.3e})")
    params = net.get_params()
    net.close()
    return params, scales, history


def evaluate(params, scales, gdot=0.01, seed=99, t0=T_START, t_end=T_END, every=5.0, n=FINE_N,
             factor=FACTOR, log=print, audit=None, projection=0):
    """L(t) of the plain fine run, of its restriction to the coarse grid, of the
    corrected coarse run and of the plain coarse run, all from the same
    restricted state at t0, with wall times.  audit = (every, window, tol)
    adds a corrected run under le_corrector_audit ("audited": its L(t), wall
    time and the audit status)."""
    import torch

    fp, cp = fine_params(gdot, n), coarse_params(gdot, n, factor)
    nc = n // factor
    fine = le.Context(fp, inputs.noise_phi0(n, n, seed, amp=0.05))
    k0 = int(round(t0 / DT))
    fine.step(k0)
    phi_c, om_c = fine.restrict(factor)
    nsamp = int(round((t_end - t0) / every))
    kf, kc = int(round(every / DT)), int(round(every / (DT * factor)))
    out = {"t": [], "fine": [], "restricted": [], "corrected": [], "coarse": []}
    sks = {"restricted": [], "corrected": [], "coarse": []}
    torch.cuda.synchronize()
    wall_fine = 0.0
    probe = le.Context(cp, np.zeros((nc, nc)))
    for i in range(nsamp):
        t_a = time.perf_counter()
        fine.step(kf)
        o, _ = fine.observables(sk=False)
        wall_fine += time.perf_counter() - t_a
        out["t"].append(o["t"])
        out["fine"].append(o["Ls"])
        pr, orr = fine.restrict(factor)
        probe.set_fields(pr, orr, (k0 + kf * (i + 1)) // factor)
        op, skp = probe.observables(sk=True)
        out["restricted"].append(op["Ls"])
        sks["restricted"].append(skp)
    fine.close()
    probe.close()
    runs = ("corrected", "coarse") + (("audited",) if audit else ())
    out["audited"] = []
    for name in runs:
        c = le.Context(cp, np.zeros((nc, nc)))
        c.set_fields(phi_c, om_c, k0 // factor)
        if name != "coarse":
            c.corrector_load(params, scales)
            c.corrector_projection(projection)
        if name == "audited":
            c.corrector_audit(*audit)
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        for i in range(nsamp):
            if name == "coarse":
                c.step(kc)
            else:
                c.step_corrected(kc)
            o, skc = c.observables(sk=True)
            out[name].append(o["Ls"])
            if name in sks:
                sks[name].append(skc)
        out["wall_" + name] = time.perf_counter() - t_a
        if name == "audited":
            fb, na, dev = c.corrector_status()
            out["audit"] = dict(every=audit[0], window=audit[1], tol=audit[2], fallback=fb,
                                audits=na, last_dev=dev)
        c.close()
    out["wall_fine"] = wall_fine
    f = np.array(out["fine"])
    fr = np.array(out["restricted"])
    out["err_mean_restriction"] = float(np.mean(np.abs(fr - f) / f))
    for name in ("corrected", "coarse"):
        e = np.abs(np.array(out[name]) - f) / f
        er = np.abs(np.array(out[name]) - fr) / fr
        out["err_mean_" + name] = float(e.mean())
        out["err_max_" + name] = float(e.max())
        out["err_mean_" + name + "_vs_restricted"] = float(er.mean())
        out["err_max_" + name + "_vs_restricted"] = float(er.max())
    # S(k) of the coarse runs against S(k) of the restricted fine field (the
    # same field seen on the coarse grid): relative L2 error per sample,
    # averaged over the samples, over the shells 1 .. nc/4 (|k| up to half the
    # coarse Nyquist), and apart over the domain band 1 .. nc/8 (the S(k) peak
    # and below) and the interface band nc/8 .. nc/2
    for name, v in sks.items():
        out["Sk_" + name] = [list(map(float, a)) for a in v]
    bands = {"": (0, nc // 4), "_low": (0, nc // 8), "_high": (nc // 8, nc // 2)}
    for suffix, (lo, hi) in bands.items():
        sr = np.array(sks["restricted"])[:, lo:hi]
        for name in ("corrected", "coarse"):
            sc = np.array(sks[name])[:, lo:hi]
            e = np.linalg.norm(sc - sr, axis=1) / np.linalg.norm(sr, axis=1)
            out["Sk" + suffix + "_err_mean_" + name] = float(e.mean())
            out["Sk" + suffix + "_err_max_" + name] = float(e.max())
    sites_fine = n * n * (t_end - t0) / DT
    out["fine_rate"] = sites_fine / wall_fine
    out["corrected_fine_equiv_rate"] = sites_fine / out["wall_corrected"]
    out["gain"] = wall_fine / out["wall_corrected"]
    if audit:
        out["audited_fine_equiv_rate"] = sites_fine / out["wall_audited"]
        out["audited_equals_corrected"] = bool(np.array_equal(out["audited"], out["corrected"]))
    log(f"corrector eval gdot={gdot}: L err mean corrected {out['err_mean_corrected']:.3f} "
        f"(vs restricted {out['err_mean_corrected_vs_restricted']:.3f}), plain coarse "
        f"{out['err_mean_coarse']:.3f} ({out['err_mean_coarse_vs_restricted']:.3f}); S(k) err "
        f"corrected {out['Sk_err_mean_corrected']:.3f} (low {out['Sk_low_err_mean_corrected']:.3f}, "
        f"high {out['Sk_high_err_mean_corrected']:.3f}), plain coarse "
        f"{out['Sk_err_mean_coarse']:.3f} (low {out['Sk_low_err_mean_coarse']:.3f}, high "
        f"{out['Sk_high_err_mean_coarse']:.3f}); gain {out['gain']:.1f}x")
    return out


def save(path, params, scales, history, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=np.asarray(params, np.float32), scales=np.asarray(scales, np.float32),
             history=np.asarray(history), meta=json.dumps(meta))


def load(path=WEIGHTS):
    with np.load(path, allow_pickle=False) as z:
        return z["params"], z["scales"], json.loads(str(z["meta"]))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=("train", "eval"))
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--weights", default=WEIGHTS)
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--seeds", type=int, nargs="*", default=[99, 98, 97])
    ap.add_argument("--gdots", type=float, nargs="*", default=[0.003, 0.01, 0.03])
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    if args.cmd == "train":
        t0 = time.time()
        xs, ts = generate_pairs(args.pairs, log=log)
        t1 = time.time()
        params, scales, hist = train(xs, ts, epochs=args.epochs, log=log)
        t2 = time.time()
        meta = dict(pairs=int(xs.shape[0]), epochs=args.epochs, data_s=t1 - t0,
                    train_s=t2 - t1, fine=FINE_N, factor=FACTOR, t_start=T_START,
                    t_end=T_END)
        save(args.out, params, scales, hist, meta)
        print(json.dumps(dict(meta, final_loss=hist[-1], first_loss=hist[0])))
    else:
        params, scales, _ = load(args.weights)
        res = []
        for g in args.gdots:
            for s in args.seeds:
                r = evaluate(params, scales, gdot=g, seed=s, log=log)
                res.append({k: v for k, v in r.items() if not isinstance(v, list)})
        print(json.dumps(res))


if __name__ == "__main__":
    main()
