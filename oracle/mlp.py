"""FP64 CPU reference of the contact-surrogate MLP (test infrastructure).

TEST INFRASTRUCTURE: used only by tests/ to check the GPU MLP kernels.

Network: x (12) -> tanh(W1 x + b1) (128) -> tanh(W2 h1 + b2) (128)
-> W3 h2 + b3 (2). The GPU multiplies BF16 operands with FP32
accumulation; this reference takes the same BF16-rounded operands
(weights and the inputs of every product) and does the arithmetic in FP64,
so the two differ only by FP32 accumulation order. BF16 rounding is
round-to-nearest-even to 8 significand bits (the upper half of an IEEE
binary32), written out below from that definition.

Loss: mean squared error over the batch and the two outputs,
L = sum((y - t)^2) / (2 n); gradients are those of L.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.atleast_1d(np.asarray(x, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out.reshape(np.shape(x))


def _identity(x):
    return np.asarray(x, np.float64)


def forward(params: dict, x: np.ndarray, rounded: bool = True):
    """Returns y [n, 2] and the activations (h1, h2) [n, 128]. With
    rounded=False the products take the operands unrounded (plain FP64)."""
    r = bf16_round if rounded else _identity
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], np.float64)
                              for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    h1 = np.tanh(r(x) @ r(W1).T + b1)
    h2 = np.tanh(r(h1) @ r(W2).T + b2)
    y = r(h2) @ r(W3).T + b3
    return y, h1, h2


def backward(params: dict, x: np.ndarray, dy: np.ndarray, rounded: bool = True):
    """Gradients of the parameters and of x for an upstream gradient dy = dL/dy.
    The products use BF16-rounded operands as the GPU kernels do (the
    upstream gradient and the activations are rounded before each product)."""
    r = bf16_round if rounded else _identity
    W1, W2, W3 = (np.asarray(params[k], np.float64) for k in ("W1", "W2", "W3"))
    _, h1, h2 = forward(params, x, rounded)
    g = {}
    g["W3"] = r(dy).T @ r(h2)
    g["b3"] = dy.sum(0)
    dh2 = r(dy) @ r(W3)
    dz2 = dh2 * (1 - h2 ** 2)
    g["W2"] = r(dz2).T @ r(h1)
    g["b2"] = dz2.sum(0)
    dh1 = r(dz2) @ r(W2)
    dz1 = dh1 * (1 - h1 ** 2)
    g["W1"] = r(dz1).T @ r(x)
    g["b1"] = dz1.sum(0)
    g["x"] = r(dz1) @ r(W1)
    return g


def loss_and_grads(params: dict, x: np.ndarray, t: np.ndarray, rounded: bool = True):
    """MSE loss and its gradients with respect to every parameter and x."""
    n = x.shape[0]
    y, _, _ = forward(params, x, rounded)
    loss = float(np.sum((y - t) ** 2) / (2 * n))
    return loss, backward(params, x, (y - t) / n, rounded)


def pack(params: dict) -> np.ndarray:
    """Parameters as the flat FP32 vector of the GPU handle (W1, b1, W2, b2, W3, b3)."""
    return np.concatenate([np.asarray(params[k], np.float32).reshape(-1)
                           for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unpack(flat: np.ndarray, n_in: int = 12, n_h: int = 128, n_out: int = 2) -> dict:
    shapes = [("W1", (n_h, n_in)), ("b1", (n_h,)), ("W2", (n_h, n_h)), ("b2", (n_h,)),
              ("W3", (n_out, n_h)), ("b3", (n_out,))]
    out, o = {}, 0
    for k, sh in shapes:
        n = int(np.prod(sh))
        out[k] = np.asarray(flat[o:o + n], np.float64).reshape(sh)
        o += n
    return out


def init_params(seed: int = 0, n_in: int = 12, n_h: int = 128, n_out: int = 2) -> dict:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) initialisation (FP32 values)."""
    rng = np.random.default_rng(seed)

    def u(shape, fan):
        b = 1.0 / np.sqrt(fan)
        return rng.uniform(-b, b, shape).astype(np.float32)
    return {"W1": u((n_h, n_in), n_in), "b1": u((n_h,), n_in),
            "W2": u((n_h, n_h), n_h), "b2": u((n_h,), n_h),
            "W3": u((n_out, n_h), n_h), "b3": u((n_out,), n_h)}
