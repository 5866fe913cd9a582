"""Physics checks of the GPU path beyond the oracle: the B = 0 absorption line
shape against Tucker's closed form (Fig. 3 parameters), run as one batched
sweep over the frequency."""
import math

import numpy as np
import pytest
import scipy.special as sp

from paper_1401_6047_amd import workloads as W
from test_oracle_pins import continuum_u, tucker

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bte():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1401_6047_amd import bte as _bte
    return _bte


def test_b0_frequency_scan_matches_tucker(bte):
    """Fig. 3 of the paper: mu = 50, E_dc = 5, E_w = 1, B = 0, omega from 0.5
    to 10.  At B = 0 the harmonics decouple and v follows the continuum
    harmonic-1 amplitude u(t) (Jacobi-Anger), so the sweep's converged A_p must
    equal the continuum periodic state averaged over the same period window
    (the batch's (p-1) L < k <= p L, dc part removed) up to O(dt^2) and the
    stopping residual; and Tucker's sum up to the window's ~|A|/L."""
    mu, E_dc, E_w, dt = 50.0, 5.0, 1.0, 2e-4
    omegas = np.linspace(0.5, 10.0, 12)
    inst = [W.Workload(f"tucker_{i}", nx=8, ny=101, phiy_min=-1.2, phiy_max=1.2, E_dc=E_dc,
                       E_w=E_w, omega=float(om), B=0.0, mu=mu, dt=dt)
            for i, om in enumerate(omegas)]
    cfg = bte.make_batch_config(8, -1.2, 1.2, dt, precision=bte.BTE_FP64, tol=1e-7,
                                min_periods=3, max_periods=200)
    b = bte.Batch(cfg, inst, autotune=False)
    b.run(log=None)
    res = b.results()
    b.close()
    ratio = sp.ive(1, mu) / sp.ive(0, mu)
    # quadrature of the thermal factor on this grid (1 to ~1e-12 here)
    y = np.linspace(-1.2, 1.2, 101)
    Q = (y[1] - y[0]) * np.sum(np.sqrt(mu / (2 * math.pi)) * np.exp(-0.5 * mu * y * y))
    for w, r in zip(inst, res):
        assert r["converged"] == 1 and r["status"] == 0, (w.omega, r)
        L = int(np.rint(2 * math.pi / (w.omega * dt)))
        P = r["periods"]
        tk = np.arange((P - 1) * L + 1, P * L + 1) * dt
        v = Q * ratio * np.imag(continuum_u(E_dc, E_w, w.omega, tk))
        A_win = (2.0 / ratio) * np.mean((v - v.mean()) * np.cos(w.omega * tk))
        assert abs(r["absorption"] - A_win) <= 2e-4 * abs(A_win) + 2e-6, (w.omega, r, A_win)
        A_t = tucker(E_dc, E_w, w.omega)
        assert abs(r["absorption"] - A_t) <= 3.0 * abs(A_t) / L + 2e-4 * abs(A_t) + 2e-6, \
            (w.omega, r["absorption"], A_t)
