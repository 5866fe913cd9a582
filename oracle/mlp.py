"""FP64 oracle of the warm-start network and of the warm-start state encoding
(test infrastructure only: imported by the tests, never by the product).

The network is not part of the paper.  It maps an instance's parameters
(E_dc, E_w, omega, B, mu) to a compressed periodic steady state of the
scheme of Sec. 3 at field phase omega t = 0 (mod 2 pi), the regime whose
current Eq. (absorption_def) averages.  Its definition, written out here in
plain numpy with float64 throughout:

    x'  = (x - shift) / scale
    H1  = gelu(x' W1^T + b1)          5 -> 256
    H2  = gelu(H1 W2^T + b2)          256 -> 256
    Y   = H2 W3^T + b3                256 -> 8192
    L   = mean over rows and outputs of (Y - out_scale c)^2

with gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2, parameters in one flat
array [W1 (256x5), b1, W2 (256x256), b2, W3 (8192x256), b3] (row-major,
[out][in]), and Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected
moments) as the update rule.

Normalisation: shift/scale are each feature's mean and population standard
deviation (scale 1 when the deviation is below 1e-6 (1 + |mean|)); out_scale is
one over the root mean square of all coefficients (1 if they are all zero).

The 64 x 128 state encoding (rows 0..31: a_n - a^(0)_n for n = 0..31; rows
32..63: b_n for n = 1..32; columns: 128 uniform phi_y points of the box,
both ends included) and its inverse use linear interpolation in phi_y;
harmonics beyond 32 decode to the equilibrium (a) and zero (b).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

N_IN, N_HID, N_OUT = 5, 256, 8192
ROWS, COLS, HARM = 64, 128, 32

SHAPES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,)))


def param_count() -> int:
    return sum(int(np.prod(s)) for _, s in SHAPES)


def offsets():
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = (o, o + size, shape)
        o += size
    return out


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    return {name: theta[a:b].reshape(shape) for name, (a, b, shape) in offsets().items()}


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    # d/dz [z Phi(z)] = Phi(z) + z phi(z)
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def normalization(features, coeffs):
    """(shift[5], scale[5], out_scale) of a data set (rows x 5, rows x 8192)."""
    x = np.asarray(features, dtype=np.float64).reshape(-1, N_IN)
    c = np.asarray(coeffs, dtype=np.float64).reshape(x.shape[0], -1)
    shift = x.mean(axis=0)
    sd = np.sqrt(((x - shift) ** 2).mean(axis=0))
    scale = np.where(sd < 1e-6 * (1.0 + np.abs(shift)), 1.0, sd)
    ms = (c * c).mean()
    out_scale = 1.0 / np.sqrt(ms) if ms > 0 else 1.0
    return shift, scale, float(out_scale)


def forward(theta, norm, features):
    """Every intermediate of the forward pass, as a dict."""
    p = unpack(theta)
    shift, scale, _ = norm
    x = np.asarray(features, dtype=np.float64).reshape(-1, N_IN)
    xn = (x - shift) / scale
    Z1 = xn @ p["W1"].T + p["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = gelu(Z2)
    Y = H2 @ p["W3"].T + p["b3"]
    return {"xn": xn, "Z1": Z1, "H1": H1, "Z2": Z2, "H2": H2, "Y": Y}


def predict(theta, norm, features):
    """Coefficients (rows x 64 x 128) in the units of the training targets."""
    Y = forward(theta, norm, features)["Y"]
    return (Y / norm[2]).reshape(-1, ROWS, COLS)


def loss_grad(theta, norm, features, coeffs):
    """(loss, gradient as one flat array in the parameter layout)."""
    p = unpack(theta)
    f = forward(theta, norm, features)
    n = f["Y"].shape[0]
    t = norm[2] * np.asarray(coeffs, dtype=np.float64).reshape(n, N_OUT)
    R = f["Y"] - t
    loss = float((R * R).mean())
    dY = 2.0 * R / (n * N_OUT)
    g = {"W3": dY.T @ f["H2"], "b3": dY.sum(axis=0)}
    dZ2 = (dY @ p["W3"]) * gelu_grad(f["Z2"])
    g["W2"] = dZ2.T @ f["H1"]
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"]) * gelu_grad(f["Z1"])
    g["W1"] = dZ1.T @ f["xn"]
    g["b1"] = dZ1.sum(axis=0)
    flat = np.concatenate([g[name].ravel() for name, _ in SHAPES])
    return loss, flat


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --------------------------------------------------------------------------
# state encoding
# --------------------------------------------------------------------------
def encode(a, b, a0):
    """64 x 128 coefficients of a whole-grid state (a, b: [n_x][n_y]) with
    equilibrium a0 ([n_x][n_y])."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nx, ny = a.shape
    u = np.arange(COLS) * (ny - 1) / (COLS - 1)      # sample positions in grid units
    grid = np.arange(ny, dtype=np.float64)
    out = np.zeros((ROWS, COLS))
    for n in range(min(HARM, nx)):
        out[n] = np.interp(u, grid, a[n] - a0[n])
    for n in range(1, min(HARM + 1, nx)):
        out[HARM + n - 1] = np.interp(u, grid, b[n])
    return out


def decode(coeffs, a0):
    """Whole-grid state (a, b) of an instance with equilibrium a0 from its
    64 x 128 coefficients."""
    a0 = np.asarray(a0, dtype=np.float64)
    c = np.asarray(coeffs, dtype=np.float64).reshape(ROWS, COLS)
    nx, ny = a0.shape
    pos = np.arange(ny) * (COLS - 1) / (ny - 1)      # grid points in sample units
    samples = np.arange(COLS, dtype=np.float64)
    a = a0.copy()
    b = np.zeros_like(a0)
    for n in range(min(HARM, nx)):
        a[n] += np.interp(pos, samples, c[n])
    for n in range(1, min(HARM + 1, nx)):
        b[n] = np.interp(pos, samples, c[HARM + n - 1])
    return a, b


# --------------------------------------------------------------------------
# element-wise rounding-error bounds of the network on the GPU
# --------------------------------------------------------------------------
# Forward error analysis of the arithmetic the GPU library performs (not of
# the network's definition above): a product C = A B over K terms whose
# operands are rounded to a format with unit roundoff u and summed in FP32
# satisfies, to first order, |fl(C) - C| <= (2u + K u32) |A| |B| element by
# element, plus |dA| |B| + |A| |dB| from errors already in the operands.
# GELU is 1.13-Lipschitz (max of Phi(z) + z phi(z)) and its derivative
# 0.80-Lipschitz (max of |phi(z) (2 - z^2)|), which carries errors through
# the activations.  The bounds below chain these through the layers in the
# order of the definition; they are worst-case (every error aligned), so an
# indexing or data-flow mistake shows up as an excess far above them while
# correct rounding stays well inside.
U_BF16 = 2.0 ** -8        # 8 significant bits
U_F32 = 2.0 ** -24
GELU_LIP = 1.13
GELU_GRAD_LIP = 0.80


def _prod_bound(A, B, dA, dB, u):
    K = A.shape[1]
    aA, aB = np.abs(A), np.abs(B)
    out = (2.0 * u + K * U_F32) * (aA @ aB)
    if dA is not None:
        out = out + dA @ aB
    if dB is not None:
        out = out + aA @ dB
    return out


def _layers(theta, norm, features, bf16):
    p = unpack(theta)
    f = forward(theta, norm, features)
    u = U_BF16 if bf16 else U_F32
    # layer 1 on the vector ALUs in FP32 (5 terms), bias add and GELU in FP32
    d_xn = 3.0 * U_F32 * np.abs(f["xn"])
    dZ1 = _prod_bound(f["xn"], p["W1"].T, d_xn, None, U_F32) + U_F32 * np.abs(f["Z1"])
    dH1 = GELU_LIP * dZ1 + 4.0 * U_F32 * np.abs(f["H1"])
    dZ2 = _prod_bound(f["H1"], p["W2"].T, dH1, None, u) + U_F32 * np.abs(f["Z2"])
    dH2 = GELU_LIP * dZ2 + 4.0 * U_F32 * np.abs(f["H2"])
    dY = _prod_bound(f["H2"], p["W3"].T, dH2, None, u) + U_F32 * np.abs(f["Y"])
    return p, f, u, {"xn": d_xn, "Z1": dZ1, "H1": dH1, "Z2": dZ2, "H2": dH2, "Y": dY}


def predict_error_bound(theta, norm, features, bf16: bool):
    """Element-wise bound of |GPU predict - predict| (rows x 64 x 128)."""
    _, f, _, d = _layers(theta, norm, features, bf16)
    Y = f["Y"] / norm[2]
    return (d["Y"] / norm[2] + U_F32 * np.abs(Y)).reshape(-1, ROWS, COLS)


def loss_grad_error_bound(theta, norm, features, coeffs, bf16: bool):
    """Element-wise bound of |GPU gradient - gradient| in the flat parameter
    layout, following the backward pass of loss_grad."""
    p, f, u, d = _layers(theta, norm, features, bf16)
    n = f["Y"].shape[0]
    t = norm[2] * np.asarray(coeffs, dtype=np.float64).reshape(n, N_OUT)
    R = f["Y"] - t
    dY = 2.0 * R / (n * N_OUT)
    e_dY = 2.0 * (d["Y"] + 2.0 * U_F32 * (np.abs(f["Y"]) + np.abs(t))) / (n * N_OUT)
    g = {"W3": _prod_bound(dY.T, f["H2"], e_dY.T, d["H2"], u),
         "b3": e_dY.sum(axis=0) + n * U_F32 * np.abs(dY).sum(axis=0)}
    A2 = dY @ p["W3"]
    e_A2 = _prod_bound(dY, p["W3"], e_dY, None, u)
    gz2 = gelu_grad(f["Z2"])
    dZ2 = A2 * gz2
    e_dZ2 = e_A2 * np.abs(gz2) + np.abs(A2) * GELU_GRAD_LIP * d["Z2"] + 4.0 * U_F32 * np.abs(dZ2)
    g["W2"] = _prod_bound(dZ2.T, f["H1"], e_dZ2.T, d["H1"], u)
    g["b2"] = e_dZ2.sum(axis=0) + n * U_F32 * np.abs(dZ2).sum(axis=0)
    A1 = dZ2 @ p["W2"]
    e_A1 = _prod_bound(dZ2, p["W2"], e_dZ2, None, u)
    gz1 = gelu_grad(f["Z1"])
    dZ1 = A1 * gz1
    e_dZ1 = e_A1 * np.abs(gz1) + np.abs(A1) * GELU_GRAD_LIP * d["Z1"] + 4.0 * U_F32 * np.abs(dZ1)
    g["W1"] = _prod_bound(dZ1.T, f["xn"], e_dZ1.T, d["xn"], U_F32)
    g["b1"] = e_dZ1.sum(axis=0) + n * U_F32 * np.abs(dZ1).sum(axis=0)
    return np.concatenate([g[name].ravel() for name, _ in SHAPES])
