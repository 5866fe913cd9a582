"""Learned warm start for parameter sweeps, end to end.

    python -m paper_1401_6047_amd.warmstart --train 32768 --test 4096 --out result.json

1. Training states: a batched sweep over seeded draws of the sweep's
   parameter distribution runs every instance to periodic convergence and
   exports its state at field phase 0 in the 64 x 128 encoding
   (``bte_batch_set_state_output``).  The training sweep may use a coarser
   grid and time step than the evaluation sweep: the encoding samples the
   same phi_y box either way, and a warm start only has to be close.
2. The network (``include/bte_mlp.h``) is trained on (parameters -> state)
   by the library's own forward/backward/Adam kernels.
3. Held-out draws at the evaluation resolution run twice, from f0 (cold) and
   from the network's prediction (warm); each run stops on its own
   period-to-period absorption criterion.  Reported: periods and wall time of
   both, and the absorption difference between them.

Everything numeric runs in ``libbte.so``; this module only sequences calls.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import bte
from . import mlp as M
from . import workloads as W


def sweep_states(instances, nx, phiy, dt, precision=bte.BTE_FP32_BULK, tol=1e-6,
                 max_periods=400, log=None, confirm=1, schedule=None):
    """Run a batched sweep to convergence; return (results, states (n,64,128)
    CUDA tensor, wall seconds)."""
    import torch
    cfg = bte.make_batch_config(nx, -phiy, phiy, dt, precision=precision, tol=tol,
                                min_periods=2, max_periods=max_periods, confirm=confirm)
    b = bte.Batch(cfg, instances, schedule=schedule)
    out = torch.zeros((len(instances), 64, 128), dtype=torch.float32, device="cuda")
    b.set_state_output(out)
    secs = b.run(log=log)
    res = b.results()
    b.close()
    return res, out, secs


def sweep(instances, nx, phiy, dt, warm=None, precision=bte.BTE_FP32_BULK, tol=1e-6,
          max_periods=400, log=None, confirm=1, schedule=None, autotune=False,
          tuning_cache=None, info=None):
    """Run a batched sweep (cold, or warm from coefficients); (results, seconds).
    With autotune the tile comes from the sweep autotuner (outside the timed
    run); `info`, a dict, receives the tile and the tuner's sample rate."""
    cfg = bte.make_batch_config(nx, -phiy, phiy, dt, precision=precision, tol=tol,
                                min_periods=2, max_periods=max_periods, confirm=confirm)
    b = bte.Batch(cfg, instances, schedule=schedule, autotune=autotune,
                  tuning_cache=tuning_cache)
    if info is not None:
        t = b.get_tuning()
        info.update(kernel=t.kernel, rows_per_wave=t.rows_per_wave,
                    waves_per_group=t.waves_per_group, tuner_cell_steps_per_s=b.tune_rate)
    b.set_warm_start(warm)
    secs = b.run(log=log)
    res = b.results()
    b.close()
    return res, secs


def coarse_draws(n, seed, nx=48, ny_by_mu=None, phiy=10.0, dt=1e-3):
    """Training draws: the sweep distribution on a 4x coarser phi_y grid and a
    10x larger time step than the sweep itself."""
    ny_by_mu = ny_by_mu or {0.25: 101, 1.0: 201, 4.0: 401}
    return W.warm_sweep_draws(n, seed, nx=nx, ny_by_mu=ny_by_mu, phi=phiy, dt=dt)


def train_network(features, states, epochs, batch=256, lr=2e-3, lr_final=2e-5, seed=0,
                  precision=M.BTE_MLP_BF16, log=None):
    net = M.Mlp(max_batch=max(batch, 256), precision=precision)
    net.set_params(W.mlp_init(seed))
    net.fit_normalization(features, states)
    t0 = time.perf_counter()
    hist = net.train(features, states, epochs=epochs, batch=batch, lr=lr, lr_final=lr_final,
                     seed=seed + 1, log=log, log_every=max(1, epochs // 10))
    return net, hist, time.perf_counter() - t0


def run(n_train, n_test, epochs, seed=W.SWEEP_SEED, train_nx=48, eval_nx=128, log=print):
    import torch
    stamp = time.perf_counter()

    def say(msg):
        if log:
            log(f"[{time.perf_counter() - stamp:7.1f} s] {msg}", flush=True)

    train = coarse_draws(n_train, seed + 1, nx=train_nx)
    say(f"training sweep: {n_train} instances, {train_nx} harmonics, coarse grid")
    tres, states, tsecs = sweep_states(train, train_nx, 10.0, train[0].dt, log=log)
    ok = np.array([r["converged"] == 1 for r in tres])
    say(f"  done in {tsecs:.1f} s; converged {ok.sum()}/{len(ok)}")
    keep = torch.as_tensor(np.nonzero(ok)[0], device="cuda")
    feats = M.features_of([w for w, k in zip(train, ok) if k])
    states = states.index_select(0, keep).contiguous()
    net, hist, secs_train = train_network(feats, states, epochs, seed=seed + 2, log=log)
    say(f"trained {epochs} epochs in {secs_train:.1f} s: loss {hist[0]:.3e} -> {hist[-1]:.3e}")

    test = W.sweep_draws(n_test, seed=seed + 3, nx=eval_nx)
    t0 = time.perf_counter()
    pred = net.predict(M.features_of(test))
    torch.cuda.synchronize()
    infer = time.perf_counter() - t0
    net.close()
    say(f"evaluation sweep: {n_test} held-out instances, cold start")
    cold, csecs = sweep(test, eval_nx, 10.0, test[0].dt, log=log)
    say(f"  cold: {csecs:.1f} s")
    warm, wsecs = sweep(test, eval_nx, 10.0, test[0].dt, warm=pred, log=log)
    say(f"  warm: {wsecs:.1f} s (+ {infer * 1e3:.1f} ms inference)")
    pc = np.array([r["periods"] for r in cold])
    pw = np.array([r["periods"] for r in warm])
    dA = np.array([abs(a["absorption"] - b["absorption"]) for a, b in zip(cold, warm)])
    cells = np.array([eval_nx * w.ny for w in test], dtype=np.float64)
    work_c = float(np.sum(cells * np.array([r["steps"] for r in cold])))
    work_w = float(np.sum(cells * np.array([r["steps"] for r in warm])))
    worst = int(np.argmax(dA))
    wt = test[worst]
    return {
        "train": {"instances": n_train, "converged": int(ok.sum()), "nx": train_nx,
                  "ny_by_mu": {"0.25": 101, "1": 201, "4": 401}, "dt": train[0].dt,
                  "sweep_s": tsecs, "epochs": epochs, "train_s": secs_train,
                  "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]},
        "test": {"instances": n_test, "nx": eval_nx,
                 "ny_by_mu": {str(k): v for k, v in W.SWEEP_NY_BY_MU.items()},
                 "dt": test[0].dt, "precision": "fp32-bulk"},
        "cold": {"periods_total": int(pc.sum()), "periods_mean": float(pc.mean()),
                 "wall_s": csecs, "converged": int(sum(r["converged"] for r in cold)),
                 "instances_per_hour": n_test / csecs * 3600,
                 "cell_steps": work_c, "cell_steps_per_s": work_c / csecs},
        "warm": {"periods_total": int(pw.sum()), "periods_mean": float(pw.mean()),
                 "wall_s": wsecs, "inference_s": infer,
                 "converged": int(sum(r["converged"] for r in warm)),
                 "instances_per_hour": n_test / (wsecs + infer) * 3600,
                 "cell_steps": work_w, "cell_steps_per_s": work_w / wsecs},
        "largest_dA": {"E_dc": wt.E_dc, "B": wt.B, "omega": wt.omega, "mu": wt.mu,
                       "cold": cold[worst], "warm": warm[worst]},
        "period_ratio": float(pw.sum() / pc.sum()),
        "speedup": float(csecs / (wsecs + infer)),
        "abs_dA_max": float(dA.max()), "abs_dA_mean": float(dA.mean()),
        "fewer_periods": int((pw < pc).sum()), "more_periods": int((pw > pc).sum()),
    }


def save_network(net, path):
    """Parameters and normalisation of a trained network (numpy .npz)."""
    np.savez(path, params=net.params().cpu().numpy(), norm=net.normalization())


def load_network(path, max_batch=512):
    d = np.load(path)          # plain arrays, no pickled objects
    net = M.Mlp(max_batch=max_batch, precision=M.BTE_MLP_BF16)
    net.set_params(d["params"])
    net.set_normalization(d["norm"])
    return net


def run_one(mode, n_test, n_train=32768, epochs=60, seed=W.SWEEP_SEED, net_path="",
            eval_nx=128, log=print, confirm=1):
    """One side of the comparison on the held-out draws: mode "cold" (from
    f0) or "warm" (network trained here on n_train coarse states, or loaded
    from net_path).  Returns per-instance results and timings."""
    import torch
    stamp = time.perf_counter()

    def say(msg):
        if log:
            log(f"[{time.perf_counter() - stamp:7.1f} s] {msg}", flush=True)

    out = {"mode": mode, "instances": n_test, "confirm": confirm}
    test = W.sweep_draws(n_test, seed=seed + 3, nx=eval_nx)
    pred, infer = None, 0.0
    if mode == "warm":
        if net_path and os.path.exists(net_path):
            net = load_network(net_path)
            out["network"] = {"loaded": net_path}
        else:
            train = coarse_draws(n_train, seed + 1)
            say(f"training sweep: {n_train} instances")
            tres, states, tsecs = sweep_states(train, train[0].nx, 10.0, train[0].dt, log=log)
            ok = [i for i, r in enumerate(tres) if r["converged"] == 1]
            keep = torch.as_tensor(ok, device="cuda")
            feats = M.features_of([train[i] for i in ok])
            net, hist, secs = train_network(feats, states.index_select(0, keep).contiguous(),
                                            epochs, seed=seed + 2, log=log)
            say(f"trained {epochs} epochs in {secs:.1f} s: loss {hist[0]:.3e} -> {hist[-1]:.3e}")
            out["network"] = {"train_instances": n_train, "converged": len(ok),
                              "sweep_s": tsecs, "epochs": epochs, "train_s": secs,
                              "loss_last_epoch": hist[-1]}
            if net_path:
                save_network(net, net_path)
        t0 = time.perf_counter()
        pred = net.predict(M.features_of(test))
        torch.cuda.synchronize()
        infer = time.perf_counter() - t0
        net.close()
    say(f"{mode} sweep of {n_test} instances")
    res, secs = sweep(test, eval_nx, 10.0, test[0].dt, warm=pred, log=log, confirm=confirm)
    say(f"  {secs:.1f} s")
    cells = [eval_nx * w.ny for w in test]
    out.update(wall_s=secs, inference_s=infer,
               cell_steps=float(sum(c * r["steps"] for c, r in zip(cells, res))),
               results=[dict(r, E_dc=w.E_dc, B=w.B, omega=w.omega, mu=w.mu)
                        for w, r in zip(test, res)])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--test", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--mode", choices=("both", "cold", "warm"), default="both",
                    help="both: train, then cold and warm sweeps; cold / warm: one side only")
    ap.add_argument("--net", default="", help="save the trained network here (warm), or load it")
    ap.add_argument("--confirm", type=int, default=1,
                    help="consecutive small period-to-period changes required to stop")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    if a.mode == "both":
        res = run(a.train, a.test, a.epochs)
    else:
        res = run_one(a.mode, a.test, a.train, a.epochs, net_path=a.net, confirm=a.confirm)
    line = json.dumps(res)
    print(line if a.mode == "both" else json.dumps({k: v for k, v in res.items() if k != "results"}),
          flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
