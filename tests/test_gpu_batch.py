"""Batched sweep (persistent schedule: one launch with a work queue; wide
schedule: one launch per pass over all running instances) with per-period
convergence, against the FP64 oracle run period by period, and against itself
across schedules, launch shapes, precision and warm starts."""
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


def oracle_periods(w, P):
    """(A_p, v_p, p L) for p = 1..P from the oracle's period-by-period run
    (the Sec. 2 absorption of each period with its mean drift velocity taken
    out, periods of L = round(T/dt) steps)."""
    pb = oracle.Problem(nx=w.nx, ny=w.ny, phiy_min=w.phiy_min, phiy_max=w.phiy_max, E_dc=w.E_dc,
                        E_w=w.E_w, omega=w.omega, B=w.B, mu=w.mu, dt=w.dt)
    return [(q.absorption, q.v_avg, q.end) for q in oracle.run_periods(pb, P)]


def make_batch(bte, inst, precision=0, tuning=None, tol=1e-6, max_periods=60, confirm=1, **kw):
    w0 = inst[0]
    cfg = bte.make_batch_config(w0.nx, w0.phiy_min, w0.phiy_max, w0.dt, precision=precision,
                                tol=tol, min_periods=2, max_periods=max_periods, confirm=confirm)
    return bte.Batch(cfg, inst, tuning=tuning, **kw)


def run_batch(bte, inst, **kw):
    b = make_batch(bte, inst, **kw)
    b.run(log=None)
    res = b.results()
    b.close()
    return res


def relerr(x, ref, floor):
    return abs(x - ref) / max(abs(ref), floor)


@pytest.fixture(scope="module")
def small():
    return W.small_sweep_draws(12, seed=20240601)


@pytest.fixture(scope="module")
def small_ref(small):
    return [oracle_periods(w, 40) for w in small]


def test_batch_fp64_matches_oracle_per_period(bte, small, small_ref):
    res = run_batch(bte, small)
    for w, r, ref in zip(small, res, small_ref):
        P = r["periods"]
        assert r["status"] == 0 and 2 <= P <= 40
        A, v, pend = ref[P - 1]
        assert r["steps"] == pend
        assert relerr(r["absorption"], A, 1e-2 * w.E_w) < 1e-10, (w.name, r, A)
        assert relerr(r["v_avg"], v, 1e-12) < 1e-10
        dA = abs(A - ref[P - 2][0])
        assert abs(r["dA"] - dA) < 1e-12
        # converged exactly when the oracle's period-to-period change is below tol,
        # and not at any earlier period
        assert r["converged"] == 1 and dA < 1e-6
        earlier = [abs(ref[p][0] - ref[p - 1][0]) for p in range(1, P - 1)]
        assert all(d >= 1e-6 for d in earlier)


def test_batch_shapes_agree_bitwise(bte, small):
    F1, F2 = bte.BTE_KERNEL_FUSED, bte.BTE_KERNEL_FUSED2
    ref = run_batch(bte, small, tuning=bte.bte_batch_tuning(F2, 25, 8, 0))
    for t in (bte.bte_batch_tuning(F1, 7, 4, 0), bte.bte_batch_tuning(F2, 3, 2, 5),
              bte.bte_batch_tuning(F1, 62, 8, 1), bte.bte_batch_tuning(F2, 58, 4, 0)):
        res = run_batch(bte, small, tuning=t)
        for a, b in zip(ref, res):
            assert a == b, (t.kernel, t.rows_per_wave, a, b)


def test_batch_fp32_bulk_within_1e5_of_oracle(bte, small, small_ref):
    res = run_batch(bte, small, precision=bte.BTE_FP32_BULK)
    for w, r, ref in zip(small, res, small_ref):
        P = r["periods"]
        A, v, pend = ref[P - 1]
        assert r["steps"] == pend
        assert abs(r["absorption"] - A) <= 1e-5
        assert abs(r["v_avg"] - v) <= 1e-5 * abs(v) + 1e-9


def test_batch_matches_single_instance_solver(bte, small):
    w = small[3]
    res = run_batch(bte, [w])
    r = res[0]
    L = int(np.rint(2.0 * math.pi / (w.omega * w.dt)))
    P = r["periods"]
    lo, hi = (P - 1) * L, P * L
    s = bte.Solver.from_workload(w)
    s.set_window(lo, hi)
    s.step(hi)
    o = s.observables()
    s.close()
    assert relerr(r["absorption"], o.absorption_cov, 1e-2 * w.E_w) < 1e-12
    assert relerr(r["v_avg"], o.v_avg, 1e-12) < 1e-12


def test_zero_warm_start_is_cold_start_and_good_warm_start_saves_periods(bte, small):
    import torch
    cold = run_batch(bte, small)
    b = make_batch(bte, small)
    b.set_warm_start(torch.zeros((len(small), 64, 128), dtype=torch.float32, device="cuda"))
    b.run(log=None)
    zero = b.results()
    b.close()
    assert zero == cold
    # warm start from the converged states of a cold run (phase 0 of the last
    # period), as exported by the sweep itself in the warm-start encoding
    b = make_batch(bte, small)
    out = torch.zeros((len(small), 64, 128), dtype=torch.float32, device="cuda")
    b.set_state_output(out)
    b.run(log=None)
    again = b.results()
    b.close()
    assert again == cold
    coeffs = out.cpu().numpy()
    # the export is the final state: check one instance against a solver run
    w, i = small[5], 5
    s = bte.Solver.from_workload(w)
    L = int(np.rint(2.0 * math.pi / (w.omega * w.dt)))
    s.step(cold[i]["periods"] * L)
    a, bb, _, _ = s.state()
    s.close()
    y = np.linspace(w.phiy_min, w.phiy_max, w.ny)
    ys = np.linspace(w.phiy_min, w.phiy_max, 128)
    a0 = oracle.equilibrium(oracle.Problem(nx=w.nx, ny=w.ny, phiy_min=w.phiy_min,
                                           phiy_max=w.phiy_max, E_dc=0, E_w=0, omega=0, B=0,
                                           mu=w.mu, dt=w.dt))
    for n in range(min(32, w.nx)):
        np.testing.assert_allclose(coeffs[i, n], np.interp(ys, y, a[n] - a0[n]), atol=1e-6)
    for n in range(1, min(33, w.nx)):
        np.testing.assert_allclose(coeffs[i, 32 + n - 1], np.interp(ys, y, bb[n]), atol=1e-6)
    b = make_batch(bte, small)
    b.set_warm_start(torch.from_numpy(coeffs).cuda())
    b.run(log=None)
    warm = b.results()
    b.close()
    # The 64 x 128 encoding itself leaves a state error of 1e-4 .. 1e-2 (linear
    # interpolation in phi_y), which the 1e-6 period criterion can still see:
    # the start saves periods in total and never costs any.  The two runs stop
    # at different periods, and a period of whole steps differs from 2 pi / w
    # by up to half a step, which moves the twice-the-frequency part of
    # v cos(w t) in A_p by up to ~|A| / K (K steps per period).
    for w, c, wr in zip(small, cold, warm):
        K = 2.0 * math.pi / (w.omega * w.dt)
        assert wr["converged"] == 1
        assert wr["periods"] <= c["periods"]
        assert abs(wr["absorption"] - c["absorption"]) < 1e-6 + 2.0 * abs(c["absorption"]) / K
    assert sum(w["periods"] for w in warm) < sum(c["periods"] for c in cold)


def test_batch_confirm_requires_consecutive_small_changes(bte, small, small_ref):
    """With confirm = 2 an instance stops at the first period p whose change
    and the previous period's change are both below tol (oracle periods)."""
    res = run_batch(bte, small, confirm=2)
    for w, r, ref in zip(small, res, small_ref):
        d = [abs(ref[p][0] - ref[p - 1][0]) for p in range(1, len(ref))]   # d[k] = |A_{k+2} - A_{k+1}|
        want = next(p + 2 for p in range(1, len(d)) if d[p] < 1e-6 and d[p - 1] < 1e-6)
        assert r["converged"] == 1 and r["periods"] == want, (w.name, r, want)
        A, v, pend = ref[want - 1]
        assert relerr(r["absorption"], A, 1e-2 * w.E_w) < 1e-10


def test_wide_schedule_matches_persistent_bitwise(bte, small, small_ref):
    """The wide schedule (one launch per pass over all running instances, one
    state slot per instance) runs the same steps, sums and stopping rule:
    identical results in FP64 and FP32 bulk, across tile shapes, with warm
    starts and state export; and against the oracle per period."""
    import torch
    F1, F2, WIDE = bte.BTE_KERNEL_FUSED, bte.BTE_KERNEL_FUSED2, bte.BTE_BATCH_WIDE
    # (FP32 bulk rounds the stored state once per pass, so the one- and
    # two-step forms differ there; each wide run is compared with the
    # persistent run of the same form)
    for precision in (0, bte.BTE_FP32_BULK):
        for kernel, R, wpg in ((F2, 25, 8), (F1, 7, 4), (F2, 58, 2)):
            ref = run_batch(bte, small, precision=precision,
                            tuning=bte.bte_batch_tuning(kernel, 25, 8, 0))
            res = run_batch(bte, small, precision=precision,
                            tuning=bte.bte_batch_tuning(kernel, R, wpg, 0, WIDE))
            for a, b in zip(ref, res):
                assert a == b, (precision, kernel, R, wpg, a, b)
    res = run_batch(bte, small, tuning=bte.bte_batch_tuning(F2, 25, 4, 0, WIDE))
    for w, r, ref in zip(small, res, small_ref):
        A, v, pend = ref[r["periods"] - 1]
        assert r["steps"] == pend and r["converged"] == 1
        assert relerr(r["absorption"], A, 1e-2 * w.E_w) < 1e-10
    # warm start and state export, twice in a row on one handle
    outs = []
    for schedule in (0, WIDE):
        b = make_batch(bte, small, tuning=bte.bte_batch_tuning(F2, 25, 8, 0, schedule))
        out = torch.zeros((len(small), 64, 128), dtype=torch.float32, device="cuda")
        b.set_state_output(out)
        b.run(log=None)
        first = b.results()
        warm = out.clone()
        b.set_warm_start(warm)
        b.run(log=None)
        second = b.results()
        b.close()
        outs.append((first, second, out.cpu().numpy(), warm.cpu().numpy()))
    (f0, s0, o0, w0), (f1, s1, o1, w1) = outs
    assert f0 == f1 and s0 == s1
    np.testing.assert_array_equal(o0, o1)
    np.testing.assert_array_equal(w0, w1)
    assert sum(r["periods"] for r in s1) < sum(r["periods"] for r in f1)


def test_wide_schedule_advance_in_slices(bte, small):
    """bte_batch_advance drives the same sweep in slices; the persistent
    schedule refuses it."""
    F2, WIDE = bte.BTE_KERNEL_FUSED2, bte.BTE_BATCH_WIDE
    ref = run_batch(bte, small, tuning=bte.bte_batch_tuning(F2, 25, 8, 0, WIDE))
    b = make_batch(bte, small, tuning=bte.bte_batch_tuning(F2, 25, 8, 0, WIDE))
    left, calls = len(small), 0
    while left:
        left = bte.bte_batch_advance(b.handle, 1)
        calls += 1
        assert 0 <= left <= len(small)
    assert calls > 1 and b.results() == ref
    b.close()
    p = make_batch(bte, small, tuning=bte.bte_batch_tuning(F2, 25, 8, 0))
    with pytest.raises(bte.BteError) as ei:
        bte.bte_batch_advance(p.handle, 1)
    assert ei.value.status == bte.BTE_ESTATE
    p.close()


def test_wide_schedule_period_cap_and_repeat_runs(bte, small):
    """An unreachable tolerance stops every instance at max_periods without
    convergence, in both schedules alike; a wide handle run twice gives the
    same results."""
    F2, WIDE = bte.BTE_KERNEL_FUSED2, bte.BTE_BATCH_WIDE
    res = {}
    for schedule in (bte.BTE_BATCH_PERSISTENT, WIDE):
        b = make_batch(bte, small, tol=1e-300, max_periods=3,
                       tuning=bte.bte_batch_tuning(F2, 58, 4, 0, schedule))
        b.run(log=None)
        first = b.results()
        b.run(log=None)
        assert b.results() == first
        b.close()
        res[schedule] = first
    assert res[WIDE] == res[bte.BTE_BATCH_PERSISTENT]
    for w, r in zip(small, res[WIDE]):
        L = int(np.rint(2.0 * math.pi / (w.omega * w.dt)))
        assert r["converged"] == 0 and r["periods"] == 3 and r["steps"] == 3 * L


def test_sweep_autotuner_picks_a_legal_shape_and_caches_it(bte, small, tmp_path):
    """bte_batch_tune times a sample of the batch for each candidate tile and
    returns one of them; the same (N_x, N_y set, precision) comes back from
    the cache without measuring; a batch run with the tuned tile gives the
    same FP64 results as with the default tile (every form and shape rounds
    alike in FP64); the JSON cache of the binding round-trips."""
    import time
    w0 = small[0]
    cfg = bte.make_batch_config(w0.nx, w0.phiy_min, w0.phiy_max, w0.dt, precision=0, tol=1e-6,
                                min_periods=2, max_periods=60)
    t, rate = bte.bte_batch_tune(cfg, small, use_cache=False)
    print(f"tuned: kernel {t.kernel} R{t.rows_per_wave} W{t.waves_per_group}, "
          f"{rate / 1e9:.1f} G cell-steps/s", flush=True)
    assert t.kernel in (bte.BTE_KERNEL_FUSED, bte.BTE_KERNEL_FUSED2)
    assert t.waves_per_group in (2, 4, 8) and t.schedule == bte.BTE_BATCH_WIDE
    assert any(t.rows_per_wave == -(-w0.nx // c) for c in range(1, 9))
    assert rate > 0
    t0 = time.perf_counter()
    t2, rate2 = bte.bte_batch_tune(cfg, list(reversed(small)))
    assert time.perf_counter() - t0 < 0.5
    assert (t2.kernel, t2.rows_per_wave, t2.waves_per_group) == \
        (t.kernel, t.rows_per_wave, t.waves_per_group) and rate2 == rate
    ref = run_batch(bte, small, precision=0)
    path = str(tmp_path / "tune.json")
    b = bte.Batch(cfg, small, autotune=True, tuning_cache=path)
    got_t = b.get_tuning()
    b.run(log=None)
    got = b.results()
    b.close()
    assert (got_t.kernel, got_t.rows_per_wave, got_t.waves_per_group) == \
        (t.kernel, t.rows_per_wave, t.waves_per_group)
    for x, y in zip(got, ref):
        assert x["absorption"] == y["absorption"] and x["periods"] == y["periods"]
    b2 = bte.Batch(cfg, small, autotune=True, tuning_cache=path)
    assert b2.tune_rate == pytest.approx(rate)
    b2.close()


def test_sweep_autotuner_second_stage_on_a_batch_larger_than_its_sample(bte):
    """A batch of more than 128 instances takes the tuner's second stage (the
    three fastest candidates re-timed on a sample as large as the batch): the
    pick is still a legal tile, is cached, and gives the default tile's FP64
    results instance by instance."""
    inst = W.small_sweep_draws(300, seed=20240611)
    w0 = inst[0]
    cfg = bte.make_batch_config(w0.nx, w0.phiy_min, w0.phiy_max, w0.dt, precision=0, tol=1e-6,
                                min_periods=2, max_periods=60)
    t, rate = bte.bte_batch_tune(cfg, inst, use_cache=False)
    print(f"tuned (300 instances): kernel {t.kernel} R{t.rows_per_wave} W{t.waves_per_group}, "
          f"{rate / 1e9:.1f} G cell-steps/s", flush=True)
    assert t.kernel in (bte.BTE_KERNEL_FUSED, bte.BTE_KERNEL_FUSED2)
    assert t.waves_per_group in (2, 4, 8) and t.schedule == bte.BTE_BATCH_WIDE
    assert any(t.rows_per_wave == -(-w0.nx // c) for c in range(1, 9)) and rate > 0
    t2, rate2 = bte.bte_batch_tune(cfg, inst)
    assert (t2.kernel, t2.rows_per_wave, t2.waves_per_group, rate2) == \
        (t.kernel, t.rows_per_wave, t.waves_per_group, rate)
    ref = run_batch(bte, inst, precision=0)
    b = bte.Batch(cfg, inst, tuning=t)
    b.run(log=None)
    got = b.results()
    b.close()
    for x, y in zip(got, ref):
        assert x["absorption"] == y["absorption"] and x["periods"] == y["periods"]
