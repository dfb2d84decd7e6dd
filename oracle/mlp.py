"""CPU oracle of the learned configuration selector: TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's CPU-baseline leg
may import this module; the product never imports it and it imports nothing
from the product.

Not in the paper (the paper tunes its kernels by hand, Table 2). Plain
definitions in float64 numpy:

- features: 4096 (or n, if fewer) keys sampled at indices floor(i * n / m),
  one 256-bin histogram per 8-bit digit place (the paper's digit places,
  Section 1) as fractions of the sample, places past the key's range zero,
  then log2(n) / 32, key_bits / 64 and has_values;
- the network: a place encoder shared by the 8 places (256 -> 16, ReLU),
  the 8 encodings and the 3 scalars concatenated (131) -> 64 ReLU -> 64 ReLU
  -> 12 outputs, one predicted log(time / best time) per configuration;
- the loss: masked mean squared error over the configurations that apply;
- Adam (Kingma and Ba, arXiv 1412.6980, Algorithm 1) with bias correction.

Pins (tests/test_oracle_mlp.py): central finite differences of the loss for
every parameter block, the closed form of Adam's steps under a constant
gradient, weights that make the network copy chosen inputs to its outputs
(layout and orientation of every layer), ReLU cut-offs, a hand-computed loss,
and features of hand-built inputs.
"""
from __future__ import annotations

import math

import numpy as np

P, R, E, S, H1, H2, C = 8, 256, 16, 3, 64, 64, 12
U = P * E + S  # 131 inputs of the first hidden layer
FEATURES = P * R + S
SAMPLES = 4096

# (name, shape) of every parameter block, in the flattened order the library
# uses.
PARAM_SHAPES = [("We", (R, E)), ("be", (E,)), ("W1", (U, H1)), ("b1", (H1,)),
                ("W2", (H1, H2)), ("b2", (H2,)), ("W3", (H2, C)), ("b3", (C,))]
NUM_PARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def unflatten(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in PARAM_SHAPES:
        k = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel()
                           for name, _ in PARAM_SHAPES])


def features(keys: np.ndarray, begin_bit: int = 0, end_bit: int | None = None,
             has_values: bool = False) -> np.ndarray:
    """Feature vector of one input (FEATURES float64 values)."""
    key_bits = keys.dtype.itemsize * 8
    end_bit = key_bits if end_bit is None else end_bit
    n = keys.size
    m = min(n, SAMPLES)
    x = np.zeros(FEATURES, dtype=np.float64)
    places = -(-(end_bit - begin_bit) // 8)
    if m > 0:
        idx = [i * n // m for i in range(m)]
        sample = [int(keys[i]) for i in idx]
        for j in range(places):
            lo = begin_bit + 8 * j
            width = min(8, end_bit - lo)
            for k in sample:
                x[j * R + ((k >> lo) & ((1 << width) - 1))] += 1.0
        x[: P * R] /= m
    x[P * R + 0] = math.log2(n) / 32.0 if n > 0 else 0.0
    x[P * R + 1] = key_bits / 64.0
    x[P * R + 2] = 1.0 if has_values else 0.0
    return x


def relu(z):
    return np.maximum(z, 0.0)


def forward(params: dict, x: np.ndarray) -> dict:
    """Activations of a batch x (B x FEATURES)."""
    x = np.asarray(x, dtype=np.float64)
    B = x.shape[0]
    hist = x[:, : P * R].reshape(B * P, R)
    enc = relu(hist @ params["We"] + params["be"])            # (B*P, E)
    u = np.concatenate([enc.reshape(B, P * E), x[:, P * R:]], axis=1)  # (B, U)
    h1 = relu(u @ params["W1"] + params["b1"])
    h2 = relu(h1 @ params["W2"] + params["b2"])
    out = h2 @ params["W3"] + params["b3"]
    return {"hist": hist, "enc": enc, "u": u, "h1": h1, "h2": h2, "out": out}


def loss(out: np.ndarray, y: np.ndarray, mask: np.ndarray) -> float:
    """Mean of the squared errors of the entries with mask 1."""
    count = max(1.0, float(mask.sum()))
    return float((mask * (out - y) ** 2).sum() / count)


def backward(params: dict, acts: dict, y: np.ndarray, mask: np.ndarray) -> dict:
    """Gradients of loss() with respect to every parameter block."""
    count = max(1.0, float(mask.sum()))
    d_out = 2.0 * mask * (acts["out"] - y) / count
    g = {}
    g["W3"] = acts["h2"].T @ d_out
    g["b3"] = d_out.sum(axis=0)
    d_h2 = (d_out @ params["W3"].T) * (acts["h2"] > 0)
    g["W2"] = acts["h1"].T @ d_h2
    g["b2"] = d_h2.sum(axis=0)
    d_h1 = (d_h2 @ params["W2"].T) * (acts["h1"] > 0)
    g["W1"] = acts["u"].T @ d_h1
    g["b1"] = d_h1.sum(axis=0)
    d_u = d_h1 @ params["W1"].T
    B = d_u.shape[0]
    d_enc = d_u[:, : P * E].reshape(B * P, E) * (acts["enc"] > 0)
    g["We"] = acts["hist"].T @ d_enc
    g["be"] = d_enc.sum(axis=0)
    return g


def adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at step number t (1-based); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v

