"""FP64 oracle of the separability-proposal network (test infrastructure only).

Network: 32 inputs -> 64 (tanh) -> 64 (tanh) -> 1 logit; the proposal score is
the logistic sigmoid of the logit. Loss: binary cross-entropy on the logit,
averaged over the minibatch. Optimizer: Adam (bias-corrected moments).

Parameters are a dict of float64 arrays: W1 (32,64), b1 (64,), W2 (64,64),
b2 (64,), W3 (64,1), b3 (1,) -- 6,337 values. Row-major, x @ W + b.
"""
from __future__ import annotations

import numpy as np

SHAPES = [("W1", (32, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
          ("W3", (64, 1)), ("b3", (1,))]


def n_params() -> int:
    return sum(int(np.prod(s)) for _, s in SHAPES)


def init_params(seed: int) -> dict:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    g = np.random.default_rng(seed)
    out = {}
    for name, shp in SHAPES:
        fan_in = shp[0] if name.startswith("W") else {"b1": 32, "b2": 64, "b3": 64}[name]
        lim = 1.0 / np.sqrt(fan_in)
        out[name] = g.uniform(-lim, lim, shp)
    return out


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], dtype=np.float64).reshape(-1) for k, _ in SHAPES])


def unflatten(vec: np.ndarray) -> dict:
    out, o = {}, 0
    for k, shp in SHAPES:
        c = int(np.prod(shp))
        out[k] = np.asarray(vec[o:o + c], dtype=np.float64).reshape(shp)
        o += c
    return out


def forward(params: dict, x: np.ndarray) -> dict:
    """Layer by layer; returns every intermediate needed by backward."""
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ params["W1"] + params["b1"]
    h1 = np.tanh(z1)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = np.tanh(z2)
    z3 = (h2 @ params["W3"] + params["b3"]).reshape(-1)
    return {"x": x, "h1": h1, "h2": h2, "logit": z3, "score": 1.0 / (1.0 + np.exp(-z3))}


def loss(params: dict, x: np.ndarray, y: np.ndarray) -> float:
    """Mean binary cross-entropy of sigmoid(logit) against labels y in {0,1}:
    log(1 + e^z) - y z, written in its overflow-free form."""
    z = forward(params, x)["logit"]
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(np.maximum(z, 0.0) - y * z + np.log1p(np.exp(-np.abs(z)))))


def backward(params: dict, x: np.ndarray, y: np.ndarray) -> dict:
    """Gradient of `loss` by the chain rule, layer by layer."""
    f = forward(params, x)
    y = np.asarray(y, dtype=np.float64)
    B = f["x"].shape[0]
    dz3 = ((f["score"] - y) / B).reshape(-1, 1)
    g = {"W3": f["h2"].T @ dz3, "b3": dz3.sum(axis=0)}
    dh2 = dz3 @ params["W3"].T
    dz2 = dh2 * (1.0 - f["h2"] ** 2)
    g["W2"] = f["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ params["W2"].T
    dz1 = dh1 * (1.0 - f["h1"] ** 2)
    g["W1"] = f["x"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(params: dict, grads: dict, m: dict, v: dict, step: int,
              lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8) -> None:
    """One Adam update in place; `step` counts from 1."""
    for k, _ in SHAPES:
        m[k] = b1 * m[k] + (1.0 - b1) * grads[k]
        v[k] = b2 * v[k] + (1.0 - b2) * grads[k] ** 2
        mh = m[k] / (1.0 - b1 ** step)
        vh = v[k] / (1.0 - b2 ** step)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
