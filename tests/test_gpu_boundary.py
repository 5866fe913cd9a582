"""Boundary behaviour of the solver's C ABI on the GPU: the resolution
diagnostics of bte_obs against the oracle, the device-side stability flag
(no bte_observables call needed for bte_step to refuse work), and the
period stopping rule bte_run_periods against the oracle run period by
period."""
import math

import numpy as np
import pytest

import oracle
from paper_1401_6047_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bte():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1401_6047_amd import bte as _bte
    return _bte


def problem(w):
    return oracle.Problem(nx=w.nx, ny=w.ny, phiy_min=w.phiy_min, phiy_max=w.phiy_max,
                          E_dc=w.E_dc, E_w=w.E_w, omega=w.omega, B=w.B, mu=w.mu, dt=w.dt,
                          alpha=w.alpha)


@pytest.mark.parametrize("nx,ny,precision", [(2, 3, 0), (9, 119, 0), (64, 250, 0),
                                              (40, 333, 1), (128, 1001, 0)])
def test_resolution_diagnostics_match_oracle(bte, nx, ny, precision):
    w = W.random_params(300 + nx + ny, nx=nx, ny=ny, phi=6.0, dt=2e-3)
    w = W.Workload(w.name, nx=w.nx, ny=w.ny, phiy_min=w.phiy_min, phiy_max=w.phiy_max,
                   E_dc=w.E_dc, E_w=w.E_w, omega=w.omega, B=w.B, mu=w.mu, dt=w.dt, alpha=0.9)
    a, b = W.smooth_state(nx * 13 + ny, nx, ny, phi=6.0)
    s = bte.Solver.from_workload(w, precision=precision)
    s.set_state(a, b)
    s.step(37)
    o = s.observables()
    st = s.state()
    s.close()
    edge, top = oracle.resolution_diagnostics(problem(w), st[0], st[1])
    assert o.status == 0
    assert abs(o.edge_mass - edge) <= 1e-12 * max(edge, 1e-300) + 1e-300
    assert abs(o.top_harm_mass - top) <= 1e-12 * max(top, 1e-300)


def test_diagnostics_of_the_equilibrium(bte):
    """At f0 the edge mass is the Boltzmann tail beyond the box's edge strips
    and the top harmonics hold (almost) nothing: both as the oracle computes
    them for the same equilibrium."""
    w = W.CROSSED
    s = bte.Solver.from_workload(w)
    o = s.observables()
    st = s.state()
    s.close()
    edge, top = oracle.resolution_diagnostics(problem(w), st[0], st[1])
    assert o.edge_mass == pytest.approx(edge, rel=1e-12, abs=1e-300)
    assert o.top_harm_mass == pytest.approx(top, rel=1e-12, abs=1e-300)
    assert o.edge_mass < 1e-15 and o.top_harm_mass < 1e-30


@pytest.mark.parametrize("row,graph_steps", [(0, 48), (1, 0), (5, 16)])
def test_device_flag_stops_stepping_without_observables(bte, row, graph_steps):
    """A NaN injected by bte_set_state is caught by the device check that ends
    every graph replay or run of direct launches; once the stream has reached
    it, bte_step refuses to queue more work, with no bte_observables call."""
    import torch
    w = W.random_params(3, nx=12, ny=41, dt=2e-3)
    s = bte.Solver.from_workload(w)
    s.set_tuning(graph_steps=graph_steps)
    a, b, af, bf = s.state()
    (a if row != 1 else b)[row, 20] = np.nan
    s.set_state(a, b, af, bf, step=0)
    s.step(48)          # a NaN in row 5 reaches rows 0 and 1 within a few steps
    torch.cuda.synchronize()
    with pytest.raises(bte.BteError) as ei:
        s.step(1)
    assert ei.value.status == bte.BTE_EUNSTABLE
    # the flag is sticky until the state is replaced
    with pytest.raises(bte.BteError):
        s.step(2)
    fresh = bte.Solver.from_workload(w)
    good = fresh.state()
    fresh.close()
    s.set_state(*good, step=0)
    s.step(48)
    torch.cuda.synchronize()
    s.step(1)
    o = s.observables()
    assert o.status == 0 and o.step == 49
    s.close()


def test_finite_state_is_never_flagged(bte):
    import torch
    w = W.CROSSED
    s = bte.Solver.from_workload(w)
    s.step(960)
    torch.cuda.synchronize()
    s.step(1)
    assert s.observables().status == 0
    s.close()


@pytest.fixture(scope="module")
def small():
    return W.small_sweep_draws(6, seed=20240611)


@pytest.mark.parametrize("confirm", [1, 2])
def test_run_periods_matches_oracle_rule(bte, small, confirm):
    """bte_run_periods stops at the first period where the oracle's
    per-period absorption has changed by less than tol on `confirm`
    consecutive periods, and reports that period's absorption and mean
    drift velocity (Sec. 2 definitions over whole-step periods)."""
    tol = 1e-6
    for w in small:
        s = bte.Solver.from_workload(w)
        r = s.run_periods(tol=tol, min_periods=2, max_periods=60, confirm=confirm)
        s.close()
        P = r["periods"]
        assert r["status"] == 0 and r["converged"] == 1 and 2 <= P <= 60
        ref = oracle.run_periods(problem(w), P)
        A = [q.absorption for q in ref]
        L = oracle.period_steps(w.omega, w.dt)
        assert r["steps"] == P * L
        floor = 1e-2 * w.E_w
        assert abs(r["absorption"] - A[-1]) < 1e-10 * max(abs(A[-1]), floor)
        assert abs(r["v_avg"] - ref[-1].v_avg) < 1e-10 * abs(ref[-1].v_avg)
        # the oracle's sequence under the same rule stops at the same period
        run_ok, stop = 0, None
        for p in range(2, P + 1):
            run_ok = run_ok + 1 if abs(A[p - 1] - A[p - 2]) < tol else 0
            if run_ok >= confirm:
                stop = p
                break
        assert stop == P, (w.name, stop, P)


def test_run_periods_equals_batch_result(bte, small):
    """The single-instance stopping rule and the batched sweep's (FP64) agree."""
    w0 = small[0]
    cfg = bte.make_batch_config(w0.nx, w0.phiy_min, w0.phiy_max, w0.dt, tol=1e-6,
                                min_periods=2, max_periods=60, confirm=2)
    b = bte.Batch(cfg, small)
    b.run(log=None)
    res = b.results()
    b.close()
    for w, rb in zip(small, res):
        s = bte.Solver.from_workload(w)
        r = s.run_periods(tol=1e-6, min_periods=2, max_periods=60, confirm=2)
        s.close()
        assert r["periods"] == rb["periods"] and r["steps"] == rb["steps"]
        assert abs(r["absorption"] - rb["absorption"]) < 1e-10 * max(abs(rb["absorption"]),
                                                                    1e-2 * w.E_w)


def test_run_periods_rejects_bad_arguments(bte):
    w = W.random_params(4, nx=8, ny=41, dt=2e-3)
    s = bte.Solver.from_workload(w)
    for args in [(0.0, 2, 10, 1), (1e-6, 1, 10, 1), (1e-6, 5, 4, 1), (1e-6, 2, 10, 0)]:
        with pytest.raises(bte.BteError) as ei:
            bte.bte_run_periods(s.handle, *args)
        assert ei.value.status == bte.BTE_EINVAL
    s.close()


@pytest.mark.parametrize("nx,ny,pad", [(2, 3, 0), (17, 187, 5), (512, 8193, 71)])
def test_state_observables_of_caller_arrays(bte, nx, ny, pad):
    """bte_state_observables on strided caller arrays: norm, v_dr and the
    resolution diagnostics of the Sec. 2 definitions, against the oracle's
    formulas on the same values (and the same with the library allocating)."""
    import torch
    a, b = W.random_coeffs(nx * 3 + ny, nx, ny, decay=0.05)
    b[0] = 0.0
    ta = torch.zeros((nx, ny + pad), dtype=torch.float64, device="cuda")
    tb = torch.zeros_like(ta)
    ta[:, :ny] = torch.from_numpy(a)
    tb[:, :ny] = torch.from_numpy(b)
    lo, hi, alpha = -7.5, 7.5, 0.9496
    got = bte.state_observables(ta[:, :ny], tb[:, :ny], lo, hi, alpha).cpu().numpy()
    pb = oracle.Problem(nx=nx, ny=ny, phiy_min=lo, phiy_max=hi, E_dc=0, E_w=0, omega=1, B=0,
                        mu=1, dt=1e-3, alpha=alpha)
    dphi = (hi - lo) / (ny - 1)
    f = math.pi * math.sqrt(alpha) * dphi
    edge, top = oracle.resolution_diagnostics(pb, a, b)
    want = [2 * f * a[0].sum(), f * b[1].sum(), edge, top]
    scale = [2 * f * np.abs(a[0]).sum(), f * np.abs(b[1]).sum(), edge, top]
    for g, w_, sc in zip(got, want, scale):
        assert abs(g - w_) <= 1e-12 * sc
    # the library-allocated workspace path gives the same bits
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    bte.bte_state_observables(ta.data_ptr(), tb.data_ptr(), nx, ny, ta.stride(0), lo, hi, alpha,
                              0, 0, torch.cuda.current_stream().cuda_stream, out.data_ptr())
    assert (out.cpu().numpy() == got).all()


def test_state_observables_rejects_bad_arguments(bte):
    import torch
    a = torch.zeros((4, 10), dtype=torch.float64, device="cuda")
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    p = a.data_ptr()
    bad = [(p, p, 1, 10, 10, -1, 1, 1), (p, p, 4, 2, 10, -1, 1, 1), (p, p, 4, 10, 9, -1, 1, 1),
           (p, p, 4, 10, 10, 1, -1, 1), (p, p, 4, 10, 10, -1, 1, 0), (0, p, 4, 10, 10, -1, 1, 1)]
    for args in bad:
        with pytest.raises(bte.BteError) as ei:
            bte.bte_state_observables(*args, 0, 0, 0, out.data_ptr())
        assert ei.value.status == bte.BTE_EINVAL
    need = bte.bte_state_observables_bytes(4)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    wp = (ws.data_ptr() + 255) // 256 * 256
    with pytest.raises(bte.BteError) as ei:
        bte.bte_state_observables(p, p, 4, 10, 10, -1, 1, 1, wp, need - 8, 0, out.data_ptr())
    assert ei.value.status == bte.BTE_ENOMEM


def test_stream_copy_copies_and_validates(bte):
    """bte_stream_copy (the measurement copy): exact bytes for one unit, for
    whole 16 KiB runs plus a partial run, and for whole runs only; rejects
    overlap and misalignment."""
    import torch
    for n in (16, 4096 * 16 + 48, 3 << 20):
        src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
        dst = torch.zeros_like(src)
        bte.bte_stream_copy(src.data_ptr(), dst.data_ptr(), n, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
    buf = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    for args in [(buf.data_ptr(), buf.data_ptr() + 256, 512), (buf.data_ptr() + 8, buf.data_ptr() + 512, 256),
                 (buf.data_ptr(), buf.data_ptr() + 512, 100)]:
        with pytest.raises(bte.BteError) as ei:
            bte.bte_stream_copy(*args)
        assert ei.value.status == bte.BTE_EINVAL
