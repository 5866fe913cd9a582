"""Seeded synthetic workloads shared by the tests, the smoke check and the bench.

This module holds only input definitions: grid shapes, physical parameters,
step counts, averaging windows and seeded random draws.  It contains none of
the solver's arithmetic, so both the HIP path and the CPU oracle can be fed
from it without sharing any code of the method.

Averaging windows follow the convention used throughout: a run of
``n_end = round(P * T / dt)`` steps with ``T = 2 pi / omega`` averages over
the last ``W = round(K_p * T / dt)`` steps, i.e. steps k with
``n_end - W < k <= n_end``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int                  # harmonics kept
    ny: int                  # phi_y points (both ends included)
    phiy_min: float
    phiy_max: float
    E_dc: float
    E_w: float
    omega: float
    B: float
    mu: float
    dt: float
    alpha: float = 1.0
    n_steps: int = 0         # full run length in whole steps
    window: tuple = (0, 0)   # (lo, hi]: steps averaged
    note: str = ""

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def with_steps(self, n_steps: int, window=None) -> "Workload":
        return replace(self, n_steps=n_steps, window=window if window is not None else (0, 0))


def periods_window(omega: float, dt: float, total_periods: float, avg_periods: float):
    """(n_end, (lo, hi)) for a run of ``total_periods`` averaged over the last
    ``avg_periods`` periods of 2 pi / omega."""
    T = 2.0 * math.pi / omega
    n_end = int(round(total_periods * T / dt))
    W = int(round(avg_periods * T / dt))
    return n_end, (n_end - W, n_end)


# Esaki-Tsu check: B = 0, E_w = 0, run to t = 20 from f0.
ESAKI_TSU = Workload("esaki_tsu_64x201", nx=64, ny=201, phiy_min=-8.0, phiy_max=8.0,
                     E_dc=1.0, E_w=0.0, omega=0.0, B=0.0, mu=1.0, dt=1e-3,
                     n_steps=20000, window=(0, 0),
                     note="64 harmonics x 201 phi_y points, t = 20")

_n2, _w2 = periods_window(2.0, 1e-4, 100, 10)
# Crossed fields: 100 ac periods, absorption over the last 10.
CROSSED = Workload("crossed_128x1001", nx=128, ny=1001, phiy_min=-10.0, phiy_max=10.0,
                   E_dc=6.0, E_w=0.1, omega=2.0, B=4.0, mu=1.0, dt=1e-4,
                   n_steps=_n2, window=_w2,
                   note="128 harmonics x 1001 phi_y points, 100 periods, average over last 10")

_n5, _w5 = periods_window(3.0, 2e-5, 500, 10)
# Large low-temperature instance: 500 ac periods (last 10 averaged).
LARGE = Workload("large_512x8193", nx=512, ny=8193, phiy_min=-20.0, phiy_max=20.0,
                 E_dc=4.0, E_w=0.5, omega=3.0, B=6.0, mu=10.0, dt=2e-5,
                 n_steps=_n5, window=_w5,
                 note="512 harmonics x 8193 phi_y points, 500 periods")

# The transient of Fig. 2's parameter set (E_dc=6, B=4, mu=3), on a small box.
FIG2_SMALL = Workload("fig2_64x201", nx=64, ny=201, phiy_min=-8.0, phiy_max=8.0,
                      E_dc=6.0, E_w=0.0, omega=0.0, B=4.0, mu=3.0, dt=1e-3,
                      n_steps=1000, window=(0, 0))

# The run the paper times in its Table 1 (Sec. 7): 120 harmonics x 4000 phi_y
# points on [-6, 6], E_dc = 7, B = 4, E_w = 0.1, omega = 10, mu = 116,
# alpha = 0.9496, dt = 1e-4, t = 10.
TABLE1 = Workload("table1_120x4000", nx=120, ny=4000, phiy_min=-6.0, phiy_max=6.0,
                  E_dc=7.0, E_w=0.1, omega=10.0, B=4.0, mu=116.0, dt=1e-4, alpha=0.9496,
                  n_steps=100000, window=(0, 0),
                  note="the paper's timing workload: 120 x 4000, 1e5 steps")

WORKLOADS = {w.name: w for w in (ESAKI_TSU, CROSSED, LARGE, FIG2_SMALL, TABLE1)}


# --------------------------------------------------------------------------
# Seeded draws
# --------------------------------------------------------------------------
def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_params(seed: int, *, nx: int, ny: int, phi: float = 6.0, dt: float = 1e-3,
                  B_max: float = 5.0, E_max: float = 6.0, mu_choices=(0.5, 1.0, 3.0),
                  E_w_max: float = 1.0) -> Workload:
    """A seeded random parameter set on a symmetric box [-phi, phi]."""
    g = rng(seed)
    return Workload(f"rand{seed}_{nx}x{ny}", nx=nx, ny=ny, phiy_min=-phi, phiy_max=phi,
                    E_dc=float(g.uniform(-E_max, E_max)), E_w=float(g.uniform(0, E_w_max)),
                    omega=float(g.uniform(0.5, 4.0)), B=float(g.uniform(-B_max, B_max)),
                    mu=float(g.choice(mu_choices)), dt=dt)


def random_coeffs(seed: int, nx: int, ny: int, decay: float = 0.0):
    """Seeded dense coefficient arrays (a, b) of shape [nx, ny], standard
    normal times exp(-decay * n) in row n; row b[0] is 0."""
    g = rng(seed)
    w = np.exp(-decay * np.arange(nx))[:, None]
    a = g.standard_normal((nx, ny)) * w
    b = g.standard_normal((nx, ny)) * w
    b[0] = 0.0
    return a, b


def smooth_state(seed: int, nx: int, ny: int, *, phi: float = 6.0, width: float = 1.5,
                 n_modes: int = 4, amp: float = 0.05):
    """Seeded smooth (a, b) arrays of shape [nx, ny]: a few low harmonics with a
    Gaussian envelope in phi_y that is ~0 at the box edges.  Row b[0] is 0."""
    g = rng(seed)
    y = np.linspace(-phi, phi, ny)
    env = np.exp(-0.5 * (y / width) ** 2)
    a = np.zeros((nx, ny))
    b = np.zeros((nx, ny))
    for n in range(min(n_modes, nx)):
        ca = g.normal(size=3)
        cb = g.normal(size=3)
        poly = ca[0] + ca[1] * y / phi + ca[2] * (y / phi) ** 2
        a[n] = amp * (0.5 ** n) * poly * env
        if n >= 1:
            polyb = cb[0] + cb[1] * y / phi + cb[2] * (y / phi) ** 2
            b[n] = amp * (0.5 ** n) * polyb * env
    a[0] += 0.1 * env
    return a, b


# --------------------------------------------------------------------------
# Batched sweep draws: E_dc ~ U[0,8], B ~ U[0,8], omega ~ U[0.5,4],
# E_w = 0.1, mu in {0.25, 1, 4}; N_y chosen by mu on phi_y in [-10, 10].
# --------------------------------------------------------------------------
SWEEP_NY_BY_MU = {0.25: 401, 1.0: 801, 4.0: 1601}
SWEEP_SEED = 14016047


def sweep_draws(n: int, seed: int = SWEEP_SEED, nx: int = 128, dt: float = 1e-4):
    g = rng(seed)
    mus = np.array(sorted(SWEEP_NY_BY_MU))
    out = []
    for i in range(n):
        E_dc = float(g.uniform(0.0, 8.0))
        B = float(g.uniform(0.0, 8.0))
        omega = float(g.uniform(0.5, 4.0))
        mu = float(mus[g.integers(0, len(mus))])
        out.append(Workload(f"sweep{seed}_{i}", nx=nx, ny=SWEEP_NY_BY_MU[mu],
                            phiy_min=-10.0, phiy_max=10.0, E_dc=E_dc, E_w=0.1,
                            omega=omega, B=B, mu=mu, dt=dt))
    return out


def small_sweep_draws(n: int, seed: int, nx: int = 16, ny_choices=(41, 61, 81),
                      phi: float = 6.0, dt: float = 2e-3):
    """Seeded small instances with uneven N_y for batch parity tests (the same
    draw shape as the sweep, on grids the CPU oracle runs in well under a
    second each)."""
    g = rng(seed)
    out = []
    for i in range(n):
        out.append(Workload(f"small{seed}_{i}", nx=nx, ny=int(ny_choices[g.integers(0, len(ny_choices))]),
                            phiy_min=-phi, phiy_max=phi, E_dc=float(g.uniform(0.0, 4.0)),
                            E_w=0.1, omega=float(g.uniform(1.5, 4.0)), B=float(g.uniform(0.0, 3.0)),
                            mu=float(g.choice([1.0, 2.0])), dt=dt))
    return out


# --------------------------------------------------------------------------
# Warm-start network: seeded initial parameters (flat, in the layout
# W1 [256][5], b1, W2 [256][256], b2, W3 [8192][256], b3).  Weights are drawn
# N(0, 1/fan_in), biases start at zero.
# --------------------------------------------------------------------------
MLP_SHAPES = ((256, 5), (256,), (256, 256), (256,), (8192, 256), (8192,))


def mlp_init(seed: int, weight_gain: float = 1.0) -> np.ndarray:
    g = rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            parts.append(g.normal(0.0, weight_gain / math.sqrt(shape[1]), size=shape).ravel())
        else:
            parts.append(np.zeros(shape[0]))
    return np.concatenate(parts).astype(np.float32)


def warm_sweep_draws(n: int, seed: int, nx: int = 24, ny_by_mu=None, phi: float = 8.0,
                     dt: float = 2e-3):
    """Seeded instances with the sweep's parameter distribution (E_dc, B ~
    U[0,8], omega ~ U[0.5,4], E_w = 0.1, mu in {0.25, 1, 4}) on reduced grids,
    for training and testing the warm start quickly."""
    ny_by_mu = ny_by_mu or {0.25: 81, 1.0: 121, 4.0: 161}
    g = rng(seed)
    mus = np.array(sorted(ny_by_mu))
    out = []
    for i in range(n):
        E_dc = float(g.uniform(0.0, 8.0))
        B = float(g.uniform(0.0, 8.0))
        omega = float(g.uniform(0.5, 4.0))
        mu = float(mus[g.integers(0, len(mus))])
        out.append(Workload(f"warm{seed}_{i}", nx=nx, ny=int(ny_by_mu[mu]), phiy_min=-phi,
                            phiy_max=phi, E_dc=E_dc, E_w=0.1, omega=omega, B=B, mu=mu, dt=dt))
    return out
