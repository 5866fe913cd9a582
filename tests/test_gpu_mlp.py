"""Warm-start network on the GPU against the FP64 oracle of the network, and
the gain the trained network brings to the sweep.

Tolerances.  Element by element, every output and gradient entry must lie
within the first-order rounding-error bound of the arithmetic the library
performs (operands rounded to BF16 or FP32, FP32 accumulation; the oracle's
predict_error_bound and loss_grad_error_bound, themselves checked against a
CPU emulation of that rounding).  Per row of outputs and per parameter
tensor, the relative error must also stay within 1e-2 in the BF16 mode and
1e-5 in the FP32 mode.
"""
import math

import numpy as np
import pytest

from oracle import mlp as omlp
from paper_1401_6047_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1401_6047_amd import mlp
    return mlp


def _data(seed, n):
    ws = W.warm_sweep_draws(n, seed)
    x = np.array([[w.E_dc, w.E_w, w.omega, w.B, w.mu] for w in ws], dtype=np.float32)
    g = W.rng(seed + 1)
    # smooth targets that depend on the features, of the coefficient scale
    base = g.normal(size=(5, 8192)) * 1e-3
    c = (np.tanh(x / 4.0) @ base + 1e-4 * g.normal(size=(n, 8192))).astype(np.float32)
    return x, c


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _oracle_norm(x, c):
    return omlp.normalization(x.astype(np.float64), c.astype(np.float64))


def test_normalization_matches_oracle(M):
    x, c = _data(11, 300)
    net = M.Mlp(max_batch=64, precision=M.BTE_MLP_FP32)
    net.fit_normalization(x, c)
    got = net.normalization()
    shift, scale, out_scale = _oracle_norm(x, c)
    np.testing.assert_allclose(got[:5], shift, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(got[5:10], scale, rtol=1e-6)
    np.testing.assert_allclose(got[10], out_scale, rtol=1e-6)
    net.close()


def _within_bound(got, want, bound, what):
    err = np.abs(np.asarray(got, np.float64) - want)
    worst = float((err / np.maximum(bound, 1e-300)).max())
    print(f"{what}: max |err| / bound = {worst:.3g}, max |err| = {err.max():.3e}", flush=True)
    bad = np.argwhere(err > bound)
    assert bad.size == 0, (what, bad[:5].tolist(), worst)


@pytest.mark.parametrize("precision,tol", [(1, 1e-5), (0, 1e-2)], ids=["fp32", "bf16"])
@pytest.mark.parametrize("n", [37, 64, 150])
def test_forward_matches_oracle(M, precision, tol, n):
    x, c = _data(12, n)
    theta = W.mlp_init(13)
    theta[omlp.offsets()["b3"][0]:] = W.rng(14).normal(size=8192) * 0.1   # nonzero output bias
    net = M.Mlp(max_batch=64, precision=precision)   # n = 150: three chunks, ragged tail
    net.set_params(theta)
    net.fit_normalization(x, c)
    got = net.predict(x).cpu().numpy()
    norm = _oracle_norm(x, c)
    th, xf = theta.astype(np.float64), x.astype(np.float64)
    want = omlp.predict(th, norm, xf)
    bound = omlp.predict_error_bound(th, norm, xf, bf16=(precision == M.BTE_MLP_BF16))
    _within_bound(got, want, bound, f"forward n={n}")
    worst = max(_rel(got[i], want[i]) for i in range(n))
    print(f"forward n={n}: worst row-wise relative error {worst:.3e}", flush=True)
    assert worst <= tol
    net.close()


@pytest.mark.parametrize("precision,tol", [(1, 1e-5), (0, 1e-2)], ids=["fp32", "bf16"])
@pytest.mark.parametrize("n", [37, 128])
def test_gradient_matches_oracle(M, precision, tol, n):
    x, c = _data(15, n)
    theta = W.mlp_init(16)
    net = M.Mlp(max_batch=128, precision=precision)
    net.set_params(theta)
    net.fit_normalization(x, c)
    loss, grad = net.loss_grad(x, c)
    grad = grad.cpu().numpy()
    norm = _oracle_norm(x, c)
    th, xf, cf = theta.astype(np.float64), x.astype(np.float64), c.astype(np.float64)
    oloss, ograd = omlp.loss_grad(th, norm, xf, cf)
    assert abs(loss - oloss) <= tol * oloss
    bound = omlp.loss_grad_error_bound(th, norm, xf, cf, bf16=(precision == M.BTE_MLP_BF16))
    for name, (a, b, _) in omlp.offsets().items():
        _within_bound(grad[a:b], ograd[a:b], bound[a:b], f"gradient {name} n={n}")
        r = _rel(grad[a:b], ograd[a:b])
        print(f"gradient {name} n={n}: relative error {r:.3e}", flush=True)
        assert r <= tol, (name, r)
    net.close()


def test_index_gather_is_the_same_as_gathered_rows(M):
    x, c = _data(17, 200)
    idx = W.rng(18).permutation(200)[:77].astype(np.int32)
    net = M.Mlp(max_batch=128, precision=M.BTE_MLP_BF16)
    net.set_params(W.mlp_init(19))
    net.fit_normalization(x, c)
    l1, g1 = net.loss_grad(x, c, index=idx)
    l2, g2 = net.loss_grad(x[idx], c[idx])
    assert l1 == l2
    assert bool((g1 == g2).all())
    net.close()


def test_adam_step_matches_oracle(M):
    x, c = _data(20, 64)
    theta = W.mlp_init(21)
    net = M.Mlp(max_batch=64, precision=M.BTE_MLP_FP32)
    net.set_params(theta)
    net.fit_normalization(x, c)
    lr = 1e-3
    _, g = net.loss_grad(x, c)
    g = g.cpu().numpy().astype(np.float64)
    net.train_step(x, c, lr)
    got = net.params().cpu().numpy()
    # the update from the GPU's own gradient: Adam's arithmetic alone
    want, m, v = omlp.adam_step(theta.astype(np.float64), g, 0.0 * g, 0.0 * g, 1, lr)
    np.testing.assert_allclose(got, want, atol=2e-7 * lr / 1e-3 + 1e-7)
    # and the step moves every parameter with a non-negligible gradient by lr
    big = np.abs(g) > 1e-4
    np.testing.assert_allclose(np.abs(got - theta)[big], lr, rtol=1e-3)
    net.close()


def test_training_fits_a_smooth_map(M):
    x, c = _data(22, 512)
    net = M.Mlp(max_batch=256, precision=M.BTE_MLP_BF16)
    net.set_params(W.mlp_init(23))
    net.fit_normalization(x, c)
    hist = net.train(x, c, epochs=60, batch=128, lr=2e-3, lr_final=1e-4, seed=24)
    assert hist[-1] < 0.05 * hist[0], hist[::10]
    net.close()


def test_trained_warm_start_saves_periods_over_cold_start(M):
    """Train on steady states the sweep itself produces (reduced grids), then
    start held-out instances from the prediction: the sweep still stops on its
    own criterion, and needs fewer periods in total for the same absorption."""
    import torch
    from paper_1401_6047_amd import bte
    train = W.warm_sweep_draws(2048, seed=31)
    test = W.warm_sweep_draws(64, seed=32)
    w0 = train[0]
    cfg = bte.make_batch_config(w0.nx, w0.phiy_min, w0.phiy_max, w0.dt,
                                precision=bte.BTE_FP32_BULK, tol=1e-6, min_periods=2,
                                max_periods=400)
    b = bte.Batch(cfg, train, autotune=False)
    states = torch.zeros((len(train), 64, 128), dtype=torch.float32, device="cuda")
    b.set_state_output(states)
    b.run(log=None)
    tr = b.results()
    b.close()
    bad = [(w, r) for w, r in zip(train, tr) if r["converged"] != 1]
    for w, r in bad[:10]:
        print(f"\nnot converged: E_dc {w.E_dc:.3f} B {w.B:.3f} omega {w.omega:.3f} mu {w.mu} "
              f"ny {w.ny}: {r}")
    assert all(r["status"] == 0 for r in tr)
    assert len(bad) <= 0.05 * len(train)
    keep = [i for i, r in enumerate(tr) if r["converged"] == 1]
    x = M.features_of([train[i] for i in keep])
    states = states[torch.as_tensor(keep, device="cuda")].contiguous()
    net = M.Mlp(max_batch=256, precision=M.BTE_MLP_BF16)
    net.set_params(W.mlp_init(33))
    net.fit_normalization(x, states)
    hist = net.train(x, states, epochs=150, batch=128, lr=2e-3, lr_final=2e-5, seed=34)
    assert hist[-1] < 0.1 * hist[0]
    pred = net.predict(M.features_of(test))
    net.close()

    def sweep(warm):
        bb = bte.Batch(cfg, test, autotune=False)
        bb.set_warm_start(warm)
        secs = bb.run(log=None)
        r = bb.results()
        bb.close()
        return r, secs

    cold, _ = sweep(None)
    warm, _ = sweep(pred)
    both = [i for i in range(len(test)) if cold[i]["converged"] == 1 and warm[i]["converged"] == 1]
    assert len(both) >= 0.9 * len(test)
    pc = sum(cold[i]["periods"] for i in both)
    pw = sum(warm[i]["periods"] for i in both)
    print(f"\nperiods to convergence over {len(test)} held-out instances: cold {pc}, "
          f"warm {pw} ({pw / pc:.3f}); final training loss {hist[-1]:.3e}")
    assert pw < 0.95 * pc
    # same attractor, each run judged by its own 1e-6 criterion, up to the
    # ~|A| / K difference of period windows of whole steps (K steps per period)
    for i in both:
        K = 2.0 * math.pi / (test[i].omega * test[i].dt)
        tol = 1e-5 + 2.0 * abs(cold[i]["absorption"]) / K
        assert abs(cold[i]["absorption"] - warm[i]["absorption"]) < tol


def test_out_of_range_rows_enter_as_zero_gradient_rows(M):
    """An index outside the data set is not read: it counts in n but adds
    nothing, so loss and gradient are those of the valid rows times n_valid/n."""
    x, c = _data(40, 100)
    valid = W.rng(41).permutation(100)[:30].astype(np.int32)
    idx = np.concatenate([valid, np.array([-1, 100, 12345], dtype=np.int32)])
    net = M.Mlp(max_batch=64, precision=M.BTE_MLP_FP32)
    net.set_params(W.mlp_init(42))
    net.fit_normalization(x, c)
    l_all, g_all = net.loss_grad(x, c, index=idx)
    l_val, g_val = net.loss_grad(x, c, index=valid)
    f = len(valid) / len(idx)
    assert abs(l_all - f * l_val) <= 1e-6 * l_val
    np.testing.assert_allclose(g_all.cpu().numpy(), f * g_val.cpu().numpy(), rtol=1e-4,
                               atol=1e-6 * float(g_val.abs().max()))
    net.close()
