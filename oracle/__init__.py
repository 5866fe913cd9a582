"""FP64 CPU oracle for the superlattice BTE solver (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python
binding) never imports, links or calls anything here, and nothing here
imports the product package.

The arithmetic lives in ``bte_oracle.c`` (plain C, FP64, OpenMP over phi_y);
this module only marshals numpy arrays into it.  ``build()`` compiles it with
gcc.  See the header of ``bte_oracle.c`` for what is computed and which
passages of the paper each part follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bte_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# No -march=native: the library is built here and may run on another host.
# -ffp-contract=off keeps every product and sum rounded as written.
CFLAGS = ["-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` and return its path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("phiy_min", ctypes.c_double), ("phiy_max", ctypes.c_double),
        ("E_dc", ctypes.c_double), ("E_w", ctypes.c_double),
        ("omega", ctypes.c_double), ("B", ctypes.c_double),
        ("mu", ctypes.c_double), ("alpha", ctypes.c_double),
        ("dt", ctypes.c_double), ("n_threads", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_bessel_ratios.argtypes = [ctypes.c_double, ctypes.c_int32, dp]
        lib.oracle_bessel_ratios.restype = ctypes.c_int
        lib.oracle_run.argtypes = [ctypes.POINTER(_Params), ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int32, ctypes.c_int32, dp, dp, dp, dp,
                                   ctypes.c_int64, ctypes.c_int64, dp, dp, dp]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_equilibrium.argtypes = [ctypes.POINTER(_Params), dp]
        lib.oracle_equilibrium.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Problem:
    """Grid and physical parameters of one instance (alpha defaults to 1)."""
    nx: int
    ny: int
    phiy_min: float
    phiy_max: float
    E_dc: float
    E_w: float
    omega: float
    B: float
    mu: float
    dt: float
    alpha: float = 1.0

    def _c(self, n_threads: int = 0) -> _Params:
        return _Params(self.nx, self.ny, self.phiy_min, self.phiy_max, self.E_dc,
                       self.E_w, self.omega, self.B, self.mu, self.alpha, self.dt,
                       n_threads)


def bessel_ratios(mu: float, nmax: int) -> np.ndarray:
    """I_n(mu)/I_0(mu) for n = 0..nmax."""
    out = np.zeros(nmax + 1)
    rc = _load().oracle_bessel_ratios(float(mu), int(nmax), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_bessel_ratios failed ({rc})")
    return out


def equilibrium(pb: Problem) -> np.ndarray:
    """a^(0)_{n,m} as an [nx, ny] array."""
    out = np.zeros((pb.nx, pb.ny))
    rc = _load().oracle_equilibrium(ctypes.byref(pb._c()), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_equilibrium failed ({rc})")
    return out


@dataclass
class Result:
    v: float            # v_dr at the last step
    norm: float         # normalisation at the last step
    S_v: float          # window sum of v_k
    S_vc: float         # window sum of v_k cos(omega t_k)
    K: int              # steps in the window
    v_avg: float        # S_v / K
    absorption: float   # (2 I_0/I_1) S_vc / K
    a_h: np.ndarray
    b_h: np.ndarray
    a_f: np.ndarray
    b_f: np.ndarray
    v_trace: np.ndarray | None = None
    norm_trace: np.ndarray | None = None
    step: int = 0


def run(pb: Problem, n_steps: int, *, window: tuple[int, int] = (0, 0),
        state: tuple[np.ndarray, ...] | None = None, k0: int = 0,
        trace: bool = False, n_threads: int = 0) -> Result:
    """Advance ``n_steps`` whole steps.

    ``state`` is None (start from f0 with the start-up half-step), a pair
    (a, b) of whole-grid arrays at step 0 (start-up half-step from it), or a
    4-tuple (a_h, b_h, a_f, b_f) at step ``k0`` (no start-up).  ``window`` is
    (lo, hi): steps k with lo < k <= hi enter the averages.
    """
    shape = (pb.nx, pb.ny)
    a_h = np.zeros(shape); b_h = np.zeros(shape)
    a_f = np.zeros(shape); b_f = np.zeros(shape)
    init_f0, startup = 1, 1
    if state is not None:
        init_f0 = 0
        if len(state) == 2:
            a_h[:] = state[0]; b_h[:] = state[1]
            if k0 != 0:
                raise ValueError("a 2-tuple state starts at step 0")
        elif len(state) == 4:
            a_h[:], b_h[:], a_f[:], b_f[:] = state
            startup = 0
        else:
            raise ValueError("state must be (a, b) or (a_h, b_h, a_f, b_f)")
    vt = np.zeros(max(n_steps, 1)) if trace else None
    nt = np.zeros(max(n_steps, 1)) if trace else None
    obs = np.zeros(7)
    rc = _load().oracle_run(ctypes.byref(pb._c(n_threads)), int(k0), int(n_steps), init_f0,
                            startup, _ptr(a_h), _ptr(b_h), _ptr(a_f), _ptr(b_f),
                            int(window[0]), int(window[1]), _ptr(vt), _ptr(nt), _ptr(obs))
    if rc != 0:
        raise ValueError(f"oracle_run failed ({rc})")
    return Result(v=obs[0], norm=obs[1], S_v=obs[2], S_vc=obs[3], K=int(obs[4]),
                  v_avg=obs[5], absorption=obs[6], a_h=a_h, b_h=b_h, a_f=a_f, b_f=b_f,
                  v_trace=vt[:n_steps] if trace else None,
                  norm_trace=nt[:n_steps] if trace else None, step=k0 + n_steps)


def max_threads() -> int:
    return int(_load().oracle_max_threads())
