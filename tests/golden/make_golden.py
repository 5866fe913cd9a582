"""Write stored expected values for the parity tests by running the FP64 oracle.

Only the oracle (``oracle/``) and the seeded workload definitions are used;
nothing here touches the HIP library.  Each output is a JSON file in this
directory named after the workload and step count.

    python tests/golden/make_golden.py crossed            # 128 x 1001, full 100 periods
    python tests/golden/make_golden.py large_prefix       # 512 x 8193, first 2000 steps
    python tests/golden/make_golden.py table1             # 120 x 4000, the paper's Table-1 run
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1401_6047_amd import workloads as W  # noqa: E402

SAMPLE_SEED = 20140123


def sample_indices(nx: int, ny: int, count: int = 256):
    g = W.rng(SAMPLE_SEED)
    n = g.integers(0, nx, size=count)
    # bias half of the samples towards the populated centre of the phi_y box
    m = np.where(np.arange(count) % 2 == 0, g.integers(0, ny, size=count),
                 np.clip((ny // 2 + g.normal(0, ny / 12, size=count)).astype(int), 0, ny - 1))
    n[:8] = [0, 1, 1, 2, nx - 1, 0, 1, 3]
    m[:8] = [ny // 2, ny // 2, 0, ny - 1, ny // 2, 0, ny // 3, 2 * ny // 3]
    return n.astype(int), m.astype(int)


def run_and_store(w: W.Workload, n_steps: int, window, tag: str, threads: int = 0):
    pb = oracle.Problem(nx=w.nx, ny=w.ny, phiy_min=w.phiy_min, phiy_max=w.phiy_max,
                        E_dc=w.E_dc, E_w=w.E_w, omega=w.omega, B=w.B, mu=w.mu, dt=w.dt,
                        alpha=w.alpha)
    t0 = time.time()
    r = oracle.run(pb, n_steps, window=window, n_threads=threads)
    secs = time.time() - t0
    n, m = sample_indices(w.nx, w.ny)
    out = {
        "workload": w.name,
        "params": {k: getattr(w, k) for k in ("nx", "ny", "phiy_min", "phiy_max", "E_dc",
                                               "E_w", "omega", "B", "mu", "dt", "alpha")},
        "n_steps": int(n_steps),
        "window": [int(window[0]), int(window[1])],
        "obs": {"v": r.v, "norm": r.norm, "S_v": r.S_v, "S_vc": r.S_vc, "K": r.K,
                "v_avg": r.v_avg, "absorption": r.absorption},
        "samples": {"n": n.tolist(), "m": m.tolist(),
                    "a_h": r.a_h[n, m].tolist(), "b_h": r.b_h[n, m].tolist(),
                    "a_f": r.a_f[n, m].tolist(), "b_f": r.b_f[n, m].tolist()},
        "row_sums": {"a_h0": float(r.a_h[0].sum()), "b_h1": float(r.b_h[1].sum())},
        "maxabs": {"a_h": float(np.abs(r.a_h).max()), "b_h": float(np.abs(r.b_h).max())},
        "generator": "tests/golden/make_golden.py (FP64 CPU oracle)",
        "oracle_seconds": secs,
        "oracle_threads": threads if threads > 0 else oracle.max_threads(),
    }
    path = os.path.join(HERE, f"{tag}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path} in {secs:.1f} s")


def main(argv):
    which = argv[1] if len(argv) > 1 else "crossed"
    threads = int(argv[2]) if len(argv) > 2 else 0
    if which == "crossed":
        w = W.CROSSED
        run_and_store(w, w.n_steps, w.window, f"{w.name}_full", threads)
    elif which == "large_prefix":
        w = W.LARGE
        run_and_store(w, 2000, (1000, 2000), f"{w.name}_2000", threads)
    elif which == "table1":
        # Sec. 7, Table 1: 1e5 steps (t = 10) from f0; absorption over the
        # last five ac periods of round(T/dt) steps each
        w = W.TABLE1
        L = int(np.rint(2.0 * np.pi / (w.omega * w.dt)))
        run_and_store(w, w.n_steps, (w.n_steps - 5 * L, w.n_steps), f"{w.name}_1e5", threads)
    else:
        raise SystemExit(f"unknown golden set {which}")


if __name__ == "__main__":
    main(sys.argv)
