"""Pins of the warm-start network oracle and the state encoding (CPU only).

Each check compares the oracle with something other than itself: central
finite differences of the loss, the normal CDF of scipy, closed forms of
Adam's first steps and of a network with zero weights, invariants of the
normalisation, and exact reconstruction of states the encoding represents
exactly.
"""
import numpy as np
import pytest
from scipy.special import ndtr

from oracle import mlp


def _rand_theta(seed, scale=1.0):
    g = np.random.default_rng(seed)
    parts = []
    for name, shape in mlp.SHAPES:
        fan_in = shape[1] if len(shape) == 2 else 1
        std = scale / np.sqrt(fan_in) if len(shape) == 2 else 0.1 * scale
        parts.append(g.normal(0.0, std, size=shape).ravel())
    return np.concatenate(parts)


def _data(seed, n):
    g = np.random.default_rng(seed)
    x = np.column_stack([g.uniform(0, 8, n), np.full(n, 0.1), g.uniform(0.5, 4, n),
                         g.uniform(0, 8, n), g.choice([0.25, 1.0, 4.0], n)])
    c = g.normal(0.0, 1e-3, size=(n, mlp.N_OUT))
    return x, c


def test_parameter_count_matches_architecture():
    # 5*256 + 256 + 256*256 + 256 + 256*8192 + 8192
    assert mlp.param_count() == 2172672


def test_gelu_is_z_times_normal_cdf_and_derivative_matches_differences():
    z = np.linspace(-8, 8, 1601)
    # the erf form cancels in 1 + erf(z) for z << 0: absolute error ~1e-16 there
    np.testing.assert_allclose(mlp.gelu(z), z * ndtr(z), rtol=1e-14, atol=1e-15)
    h = 1e-5
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, atol=1e-9)


def test_normalization_standardizes_features_and_targets():
    x, c = _data(1, 300)
    shift, scale, out_scale = mlp.normalization(x, c)
    xn = (x - shift) / scale
    varying = [0, 2, 3, 4]
    np.testing.assert_allclose(xn[:, varying].mean(axis=0), 0, atol=1e-12)
    np.testing.assert_allclose(xn[:, varying].std(axis=0), 1, rtol=1e-12)
    # the constant feature (E_w) keeps scale 1 and maps to 0
    assert scale[1] == 1.0 and np.all(np.abs(xn[:, 1]) < 1e-14)
    np.testing.assert_allclose(np.sqrt(np.mean((out_scale * c) ** 2)), 1.0, rtol=1e-12)
    assert mlp.normalization(x, np.zeros_like(c))[2] == 1.0


def test_gradient_matches_central_differences():
    x, c = _data(2, 6)
    norm = mlp.normalization(x, c)
    theta = _rand_theta(3)
    loss, grad = mlp.loss_grad(theta, norm, x, c)
    g = np.random.default_rng(4)
    h = 1e-6
    for name, (a, b, _) in mlp.offsets().items():
        idx = g.choice(np.arange(a, b), size=12, replace=False)
        if name == "W3":
            # also the largest entries, so the check is not only on tiny ones
            idx = np.concatenate([idx, a + np.argsort(-np.abs(grad[a:b]))[:4]])
        for i in idx:
            tp = theta.copy()
            tm = theta.copy()
            tp[i] += h
            tm[i] -= h
            fd = (mlp.loss_grad(tp, norm, x, c)[0] - mlp.loss_grad(tm, norm, x, c)[0]) / (2 * h)
            # rounding of the O(1) loss over 2h: ~1e-10; truncation: ~h^2
            assert abs(fd - grad[i]) <= 1e-6 * abs(grad[i]) + 1e-9, (name, i, fd, grad[i])


def test_zero_weights_give_the_output_bias_and_its_closed_form_gradient():
    x, c = _data(5, 9)
    norm = mlp.normalization(x, c)
    theta = np.zeros(mlp.param_count())
    o = mlp.offsets()
    b3 = np.random.default_rng(6).normal(size=mlp.N_OUT)
    theta[o["b3"][0]:o["b3"][1]] = b3
    pred = mlp.predict(theta, norm, x).reshape(9, -1)
    np.testing.assert_allclose(pred, np.tile(b3 / norm[2], (9, 1)), rtol=1e-15)
    loss, grad = mlp.loss_grad(theta, norm, x, c)
    t = norm[2] * c
    np.testing.assert_allclose(loss, np.mean((b3 - t) ** 2), rtol=1e-14)
    np.testing.assert_allclose(grad[o["b3"][0]:o["b3"][1]],
                               2.0 * (b3 - t).sum(axis=0) / (9 * mlp.N_OUT), rtol=1e-12)
    # every other gradient vanishes: the hidden activations do not reach Y
    assert np.all(grad[o["W3"][0]:o["W3"][1]] == 0.0)
    assert np.all(grad[:o["W3"][0]] == 0.0)


def test_adam_first_steps_move_every_parameter_by_lr_against_the_gradient_sign():
    g = np.random.default_rng(7)
    theta = g.normal(size=1000)
    grad = g.normal(size=1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    t1, m, v = mlp.adam_step(theta, grad, m, v, 1, 1e-3)
    # bias-corrected moments are g and g^2 after step 1 (and with a constant
    # gradient after step 2): the update is lr * g / (|g| + eps)
    np.testing.assert_allclose(t1 - theta, -1e-3 * grad / (np.abs(grad) + 1e-8), rtol=1e-12)
    t2, m, v = mlp.adam_step(t1, grad, m, v, 2, 1e-3)
    np.testing.assert_allclose(t2 - t1, -1e-3 * grad / (np.abs(grad) + 1e-8), rtol=1e-9)


def test_encoding_round_trip_is_exact_for_states_linear_in_phi():
    nx, ny = 40, 161
    y = np.linspace(-6, 6, ny)
    a0 = np.exp(-0.5 * y * y)[None, :] * (0.5 ** np.arange(nx))[:, None]
    a = a0.copy()
    b = np.zeros((nx, ny))
    for n in range(nx):
        a[n] += 0.01 * (n + 1) * (1.0 + 0.3 * y)
        if n >= 1:
            b[n] = 0.02 * (2.0 - 0.1 * n * y)
    c = mlp.encode(a, b, a0)
    ra, rb = mlp.decode(c, a0)
    # harmonics 0..31 (a) and 1..32 (b) come back exactly; the rest decode to
    # the equilibrium and zero
    np.testing.assert_allclose(ra[:32], a[:32], atol=1e-14)
    np.testing.assert_allclose(rb[:33], b[:33], atol=1e-14)
    np.testing.assert_array_equal(ra[32:], a0[32:])
    np.testing.assert_array_equal(rb[33:], 0.0)
    # the equilibrium itself encodes to zero
    assert np.all(mlp.encode(a0, np.zeros((nx, ny)), a0) == 0.0)


def test_encoding_samples_are_grid_values_where_the_grids_coincide():
    # n_y = 128 (or 127 k + 1) puts every sample on a grid point
    nx = 8
    g = np.random.default_rng(8)
    for ny in (128, 255):
        a0 = g.normal(size=(nx, ny))
        a = a0 + g.normal(size=(nx, ny))
        b = g.normal(size=(nx, ny))
        c = mlp.encode(a, b, a0)
        step = (ny - 1) // 127
        np.testing.assert_allclose(c[:nx], (a - a0)[:, ::step], atol=1e-14)
        np.testing.assert_allclose(c[32:32 + nx - 1], b[1:, ::step], atol=1e-14)


@pytest.mark.parametrize("n", [1, 5])
def test_predict_shape(n):
    x, c = _data(9, n)
    out = mlp.predict(_rand_theta(10), mlp.normalization(x, c), x)
    assert out.shape == (n, 64, 128)


def _bf16(a):
    """Round float64 values to bfloat16 (8 significant bits, nearest-even) by
    rounding the float32 bit pattern, the way the GPU converts operands."""
    f = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    f = (f + 0x7FFF + ((f >> 16) & 1)) & 0xFFFF0000
    return f.astype(np.uint32).view(np.float32).astype(np.float64)


def _emulated_forward(theta, norm, x, bf16):
    """The GPU's rounding model run on the CPU: layer 1 in float32, the two
    large products with operands rounded (bf16 or float32) and float32 sums."""
    p = mlp.unpack(theta)
    r = _bf16 if bf16 else (lambda a: np.asarray(a, np.float32).astype(np.float64))
    f32 = np.float32
    xn = ((x.astype(f32) - norm[0].astype(f32)) / norm[1].astype(f32)).astype(f32)
    Z1 = (xn @ p["W1"].T.astype(f32) + p["b1"].astype(f32)).astype(np.float64)
    H1 = mlp.gelu(Z1)
    Z2 = (r(H1).astype(f32) @ r(p["W2"].T).astype(f32)).astype(np.float64) + p["b2"]
    H2 = mlp.gelu(Z2)
    Y = (r(H2).astype(f32) @ r(p["W3"].T).astype(f32)).astype(np.float64) + p["b3"]
    return Y / norm[2]


@pytest.mark.parametrize("bf16", [True, False])
def test_forward_error_bound_holds_for_the_rounding_model(bf16):
    """The element-wise bound contains the error of a CPU emulation of the
    GPU's rounding (operands rounded, float32 sums) and is not vacuous: the
    emulated error reaches a visible share of it somewhere."""
    g = np.random.default_rng(5)
    theta = np.concatenate([g.normal(size=int(np.prod(s))) / np.sqrt(s[-1]) if len(s) == 2
                            else 0.1 * g.normal(size=s[0]) for _, s in mlp.SHAPES])
    x = g.normal(size=(24, 5)) * [2, 0.1, 1, 2, 1] + [4, 0.1, 2, 4, 1]
    c = g.normal(size=(24, 8192)) * 1e-3
    norm = mlp.normalization(x, c)
    want = mlp.predict(theta, norm, x).reshape(24, -1)
    got = _emulated_forward(theta, norm, x, bf16)
    bound = mlp.predict_error_bound(theta, norm, x, bf16).reshape(24, -1)
    err = np.abs(got - want)
    assert np.all(err <= bound)
    assert (err / bound).max() > (1e-2 if bf16 else 1e-4)
    # operand rounding dominates in bf16 (2 u_bf16 against 256 u_f32 of
    # float32 summation): the bf16 bounds are a few hundred times wider
    other = mlp.predict_error_bound(theta, norm, x, not bf16).reshape(24, -1)
    ratio = np.median(bound / other)
    assert (ratio > 100) if bf16 else (ratio < 1e-2)
