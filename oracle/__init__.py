"""FP64 CPU oracle for the superlattice BTE solver (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python
binding) never imports, links or calls anything here, and nothing here
imports the product package.

The arithmetic lives in ``bte_oracle.c`` (plain C, FP64, OpenMP over phi_y)
and ``characteristics.c`` (the same physics by characteristic curves, Sec. 4);
this module marshals numpy arrays into them.  Written here in numpy are
only the quadrature nodes of the equilibrium average, the absorption taken
period by period from the C oracle's drift-velocity trace, and the B = 0
continuum references (the Jacobi-Anger periodic state and Tucker's sum).
``build()`` compiles the C part with gcc.  See the header of ``bte_oracle.c`` for what is computed and which
passages of the paper each part follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "bte_oracle.c"), os.path.join(_HERE, "characteristics.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

# No -march=native: the library is built here and may run on another host.
# -ffp-contract=off keeps every product and sum rounded as written.
CFLAGS = ["-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` and return its path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", *CFLAGS, "-o", tmp, *_SRC, "-lm"]
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
        lib.oracle_characteristic_v.argtypes = [
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
            dp, dp, dp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32, dp]
        lib.oracle_characteristic_v.restype = ctypes.c_int
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


# ---------------------------------------------------------------------------
# Characteristic curves (Sec. 4): pendulum flow with exponential memory.
# ---------------------------------------------------------------------------
def equilibrium_nodes(mu: float | None, n: int = 12):
    """Nodes and weights of the average over the equilibrium distribution of
    Sec. 2 (density proportional to exp(mu cos phi_x - mu phi_y^2 / 2)).

    ``mu`` None is the zero-temperature limit: one node at the origin.
    Otherwise an n x n Gauss-Hermite product rule in units of 1/sqrt(mu):
    exact in phi_y (a Gaussian), and in phi_x the factor
    exp(mu (cos x - 1 + x^2/2)) is folded into the weights.  The phi_x rule
    ignores the periodic images of the peak, so it is meant for large mu
    (narrow peak); the nodes must stay inside |phi_x| < pi/2.
    """
    if mu is None:
        return np.zeros(1), np.zeros(1), np.ones(1)
    t, wt = np.polynomial.hermite.hermgauss(int(n))
    s = np.sqrt(2.0 / mu)
    x = s * t
    if np.abs(x).max() >= np.pi / 2:
        raise ValueError("equilibrium_nodes: peak too wide for the Gauss-Hermite rule")
    wx = wt * np.exp(mu * (np.cos(x) - 1.0 + 0.5 * x * x))
    wx /= wx.sum()
    wy = wt / wt.sum()
    X, Y = np.meshgrid(x, s * t, indexing="ij")
    return X.ravel().copy(), Y.ravel().copy(), np.outer(wx, wy).ravel().copy()


def characteristic_v(E_dc: float, E_w: float, omega: float, B: float, mu: float | None,
                     *, h: float = 0.01, tau_max: float = 36.0, nodes: int = 12,
                     n_threads: int = 0):
    """v_dr(t_i) of the periodic state on t_i = i*h', i < n, with n h' one
    field period (h' is the largest step <= h that divides the period); for
    E_w = 0 one value.  Returns (t, v)."""
    x0, y0, w = equilibrium_nodes(mu, nodes)
    if E_w != 0.0:
        period = 2.0 * np.pi / omega
        n = int(np.ceil(period / h))
        hh = period / n
    else:
        n, hh = 1, h
    v = np.zeros(n)
    rc = _load().oracle_characteristic_v(float(E_dc), float(E_w), float(omega), float(B),
                                         len(w), _ptr(x0), _ptr(y0), _ptr(w), n, hh,
                                         float(tau_max), int(n_threads), _ptr(v))
    if rc != 0:
        raise ValueError(f"oracle_characteristic_v failed ({rc})")
    return np.arange(n) * hh, v


def characteristic_absorption(E_dc: float, E_w: float, omega: float, B: float,
                              mu: float | None, **kw) -> float:
    """A = <(2 I_0/I_1) v_dr(t) cos(omega t)>_t over one period of the
    periodic state (Sec. 2); I_0/I_1 -> 1 in the zero-temperature limit.
    The period mean of a sampled periodic function is the plain mean of
    equally spaced samples."""
    t, v = characteristic_v(E_dc, E_w, omega, B, mu, **kw)
    r = 1.0 if mu is None else 1.0 / bessel_ratios(mu, 1)[1]
    return float(2.0 * r * np.mean(v * np.cos(omega * t)))


# ---------------------------------------------------------------------------
# The distribution function from its Fourier coefficients (Sec. 2).
# ---------------------------------------------------------------------------
def reconstruct(a: np.ndarray, b: np.ndarray, n_phix: int,
                cols: np.ndarray | None = None, rows: np.ndarray | None = None) -> np.ndarray:
    """f(x_j, phi_y(m)) = sum_n a_n(m) cos(n x_j) + b_n(m) sin(n x_j) (Eq.
    f_fourier) on x_j = -pi + 2 pi j / n_phix; b_0 is taken as zero.

    a, b: [N_x, N_y] arrays.  Returns [n_phix, N_y], or only the samples
    (rows[i], cols[i]) when both index arrays are given."""
    a = np.asarray(a, dtype=np.float64)
    b = np.array(b, dtype=np.float64)
    b[0] = 0.0
    n = np.arange(a.shape[0])
    if rows is not None and cols is not None:
        x = -np.pi + 2.0 * np.pi * np.asarray(rows) / n_phix
        ang = np.outer(x, n)
        return np.einsum("in,ni->i", np.cos(ang), a[:, cols]) + \
            np.einsum("in,ni->i", np.sin(ang), b[:, cols])
    x = -np.pi + 2.0 * np.pi * np.arange(n_phix) / n_phix
    ang = np.outer(x, n)
    return np.cos(ang) @ a + np.sin(ang) @ b


# ---------------------------------------------------------------------------
# Absorption period by period (Sec. 2 absorption, taken over each ac period).
# ---------------------------------------------------------------------------
def period_steps(omega: float, dt: float) -> int:
    """Whole steps per ac period: L = round(2 pi / (omega dt))."""
    return max(1, int(np.rint(2.0 * np.pi / (omega * dt))))


@dataclass
class Period:
    absorption: float   # A_p: (2 I_0/I_1) mean over the period of (v - <v>_p) cos(omega t)
    v_avg: float        # <v>_p: mean drift velocity over the period
    end: int            # last step of the period, p L
    plain: float        # (2 I_0/I_1) mean of v cos(omega t) over the same steps (no mean taken out)


def run_periods(pb: Problem, n_periods: int, *, n_threads: int = 0) -> list[Period]:
    """The oracle run period by period from f0 (start-up at step 0, phase 0 of
    the field).  Period p covers the steps (p-1) L < k <= p L, L =
    period_steps(omega, dt): windows of one length, so that the half-step by
    which L dt misses 2 pi / omega is the same in every period.  The
    absorption of a period is the Sec. 2 average of (2 I_0/I_1) v cos(omega t)
    over its steps with the period's mean drift velocity taken out first: on
    a window of exactly one period the two agree (the cosine averages to
    zero); on a window of whole steps the plain average also picks up
    <v> times the window's cosine mean, a dc leak that alternates in sign
    from period to period.  t_k = k dt; v_k from the oracle's trace."""
    L = period_steps(pb.omega, pb.dt)
    scale = 2.0 / bessel_ratios(pb.mu, 1)[1]
    out, state, k = [], None, 0
    for p in range(1, n_periods + 1):
        r = run(pb, L, state=state, k0=k, trace=True, n_threads=n_threads)
        steps = np.arange(k + 1, k + L + 1, dtype=np.float64)
        c = np.cos(pb.omega * (steps * pb.dt))
        v = r.v_trace
        vbar = float(np.mean(v))
        out.append(Period(absorption=scale * float(np.mean((v - vbar) * c)), v_avg=vbar,
                          end=k + L, plain=scale * float(np.mean(v * c))))
        state, k = (r.a_h, r.b_h, r.a_f, r.b_f), k + L
    return out


# ---------------------------------------------------------------------------
# Continuum references at B = 0 (Sec. 2 Fourier system, harmonic 1).
# ---------------------------------------------------------------------------
# At B = 0 the transport terms vanish except the field term, so the harmonics
# decouple.  For harmonic 1, w = a_1 + i b_1 obeys dw/dt = a^(0)_1 - (1 - i
# E(t)) w at every phi_y, and v_dr = pi sqrt(alpha) \int b_1 dphi_y.  With
# u = w / a^(0)_1 and the normalisation of a^(0)_1 (its phi_y integral is
# (I_1/I_0) / (pi sqrt(alpha))), v_dr = (I_1/I_0) Im u, where u solves
#     du/dt = 1 - (1 - i E(t)) u,   E(t) = E_dc + E_w cos(omega t).
# Its periodic solution follows from the Jacobi-Anger expansion
# e^{i a sin(omega t)} = sum_l J_l(a) e^{i l omega t}, a = E_w / omega.
def continuum_u(E_dc: float, E_w: float, omega: float, t, lmax: int = 30) -> np.ndarray:
    """Periodic solution u(t) = sum_{n,l} J_n(a) J_l(a) e^{i (n - l) omega t} /
    (1 - i (E_dc + l omega)) of du/dt = 1 - (1 - i E(t)) u (the harmonic-1
    amplitude at B = 0 in units of its equilibrium value)."""
    import scipy.special as sp
    t = np.asarray(t, dtype=np.float64)
    a = E_w / omega
    l = np.arange(-lmax, lmax + 1)
    J = sp.jv(l, a)
    coef_l = J / (1.0 - 1j * (E_dc + l * omega))
    ph_n = np.exp(1j * np.outer(t, l) * omega) @ J              # sum_n J_n e^{i n w t}
    ph_l = np.exp(-1j * np.outer(t, l) * omega) @ coef_l        # sum_l J_l e^{-i l w t} / (...)
    return ph_n * ph_l


def tucker_absorption(E_dc: float, E_w: float, omega: float, lmax: int = 60) -> float:
    """Period average of (2 I_0/I_1) v_dr cos(omega t) for the periodic state
    at B = 0: 2 <Im u cos(omega t)>, which the Jacobi-Anger form above sums to
    sum_l J_l(a) [J_{l+1}(a) + J_{l-1}(a)] xi(E_dc + l omega), xi(x) = x/(1+x^2),
    a = E_w/omega (Tucker's closed form as derived from the Fourier system;
    the paper prints it with an extra factor 2 I_1/I_0)."""
    import scipy.special as sp
    a = E_w / omega
    l = np.arange(-lmax, lmax + 1)
    x = E_dc + l * omega
    return float(np.sum(sp.jv(l, a) * (sp.jv(l + 1, a) + sp.jv(l - 1, a)) * x / (1.0 + x * x)))


# ---------------------------------------------------------------------------
# Resolution diagnostics of a whole-grid state.
# ---------------------------------------------------------------------------
def edge_width(ny: int) -> int:
    """phi_y points in each edge strip: max(1, ceil(N_y / 64))."""
    return max(1, -(-ny // 64))


def top_harmonics(nx: int) -> int:
    """Harmonics counted as the top of the spectrum: max(1, N_x // 8)."""
    return max(1, nx // 8)


def resolution_diagnostics(pb: Problem, a: np.ndarray, b: np.ndarray) -> tuple[float, float]:
    """(edge_mass, top_harm_mass) of the state (a, b) ([N_x, N_y] arrays).

    edge_mass: the normalisation integral of Sec. 2, 2 pi sqrt(alpha) dphi
    sum_m a_0(m), taken over |a_0| in the outer edge_width(N_y) points on each
    side of the phi_y box.  top_harm_mass: the share of the integral of f^2
    over phi_x in [-pi, pi) and the box carried by the top top_harmonics(N_x)
    harmonics; by Parseval's theorem for the Fourier series of Sec. 2 that
    integral is pi dphi sum_m [2 a_0^2 + sum_{n>=1} (a_n^2 + b_n^2)]."""
    a = np.asarray(a, dtype=np.float64)
    b = np.array(b, dtype=np.float64)
    b[0] = 0.0
    dphi = (pb.phiy_max - pb.phiy_min) / (pb.ny - 1)
    w = edge_width(pb.ny)
    edge = np.abs(a[0, :w]).sum() + np.abs(a[0, pb.ny - w:]).sum()
    edge_mass = 2.0 * np.pi * np.sqrt(pb.alpha) * dphi * edge
    h = top_harmonics(pb.nx)
    energy = a * a + b * b
    total = 2.0 * np.sum(a[0] ** 2) + np.sum(energy[1:])
    top = np.sum(energy[pb.nx - h:])
    return float(edge_mass), float(top / total) if total > 0 else 0.0
