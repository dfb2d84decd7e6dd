"""Pins of the MLP oracle (oracle/mlp.py) against things other than itself:
central finite differences, Adam's closed-form steps, weight settings that
reduce the network to reading chosen inputs, and hand-built feature inputs."""
import numpy as np
import pytest

from oracle import mlp as M


def random_case(seed, B=5):
    rng = np.random.default_rng(seed)
    params = {}
    for name, shape in M.PARAM_SHAPES:
        params[name] = rng.normal(0.0, 0.3, size=shape)
    x = np.zeros((B, M.FEATURES))
    x[:, : M.P * M.R] = rng.random((B, M.P * M.R)) / 32.0
    x[:, M.P * M.R:] = rng.random((B, M.S))
    y = rng.normal(0.0, 1.0, size=(B, M.C))
    mask = (rng.random((B, M.C)) < 0.7).astype(np.float64)
    return params, x, y, mask


def total_loss(params, x, y, mask):
    return M.loss(M.forward(params, x)["out"], y, mask)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_central_differences(seed):
    params, x, y, mask = random_case(seed)
    grads = M.backward(params, M.forward(params, x), y, mask)
    rng = np.random.default_rng(100 + seed)
    h = 1e-6
    for name, shape in M.PARAM_SHAPES:
        flat = params[name].ravel()
        picks = rng.choice(flat.size, size=min(flat.size, 40), replace=False)
        for i in picks:
            keep = flat[i]
            flat[i] = keep + h
            lp = total_loss(params, x, y, mask)
            flat[i] = keep - h
            lm = total_loss(params, x, y, mask)
            flat[i] = keep
            fd = (lp - lm) / (2 * h)
            g = grads[name].ravel()[i]
            assert abs(fd - g) <= 1e-6 + 1e-5 * abs(g), (name, i, fd, g)


def test_loss_small_example():
    out = np.array([[1.0, 2.0], [3.0, -1.0]])
    y = np.zeros((2, 2))
    mask = np.array([[1.0, 0.0], [1.0, 1.0]])
    assert M.loss(out, y, mask) == pytest.approx((1 + 9 + 1) / 3)
    assert M.loss(out, y, np.zeros((2, 2))) == 0.0


def test_adam_first_steps_closed_form():
    # With a constant gradient g, the bias-corrected moments are g and g^2 at
    # every step, so each step moves theta by -lr * g / (|g| + eps).
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    theta = np.array([1.0, 1.0, 1.0, 1.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for t in (1, 2, 3):
        new, m, v = M.adam(theta, g, m, v, t, lr=lr, eps=eps)
        np.testing.assert_allclose(new - theta, -lr * g / (np.abs(g) + eps), rtol=1e-9,
                                   atol=1e-15)
        theta = new


def test_selector_weights_read_chosen_inputs():
    """Weights that copy chosen inputs through every layer pin the layout:
    place/bin order of the histogram block, the concatenation order of the
    encodings and scalars, and the orientation of every weight matrix."""
    p = {name: np.zeros(shape) for name, shape in M.PARAM_SHAPES}
    # encoder unit k reads bin 10 + k of each place
    for k in range(M.E):
        p["We"][10 + k, k] = 1.0
    # hidden unit c of layer 1 reads: c < 8 -> place c's unit c; c = 8, 9, 10 -> scalars
    for c in range(8):
        p["W1"][c * M.E + c, c] = 1.0
    for s in range(M.S):
        p["W1"][M.P * M.E + s, 8 + s] = 1.0
    p["W2"][: M.H1, : M.H2] = np.eye(M.H1, M.H2)
    for c in range(11):
        p["W3"][c, c] = 1.0
    p["b3"][11] = 0.25
    rng = np.random.default_rng(7)
    x = np.zeros((3, M.FEATURES))
    x[:, : M.P * M.R] = rng.random((3, M.P * M.R))
    x[:, M.P * M.R:] = rng.random((3, M.S))
    out = M.forward(p, x)["out"]
    for b in range(3):
        for c in range(8):
            assert out[b, c] == x[b, c * M.R + 10 + c]
        for s in range(M.S):
            assert out[b, 8 + s] == x[b, M.P * M.R + s]
        assert out[b, 11] == 0.25


def test_relu_cuts_negative_preactivations():
    p = {name: np.zeros(shape) for name, shape in M.PARAM_SHAPES}
    p["be"][:] = -1.0  # every encoding is ReLU(-1 + 0) = 0
    p["W1"][:, :] = 1.0
    p["W3"][:, :] = 1.0
    x = np.zeros((1, M.FEATURES))
    x[0, M.P * M.R:] = [0.5, 0.25, 1.0]
    out = M.forward(p, x)["out"]
    # h1 = sum of scalars = 1.75 in every unit; h2 = ReLU(0) = 0 (W2 zero)
    assert np.all(out == 0.0)
    p["W2"][:, :] = np.eye(M.H1, M.H2)
    out = M.forward(p, x)["out"]
    assert np.allclose(out, 1.75 * M.H2)


def test_features_hand_built_inputs():
    # every key identical: each place has all its mass in one bin
    keys = np.full(5000, 0x0A0B0C0D, dtype=np.uint32)
    f = M.features(keys)
    for j, v in enumerate((0x0D, 0x0C, 0x0B, 0x0A)):
        row = f[j * M.R:(j + 1) * M.R]
        assert row[v] == 1.0 and row.sum() == 1.0
    assert not f[4 * M.R: 8 * M.R].any()  # 32-bit keys leave places 4..7 empty
    assert f[M.P * M.R:].tolist() == [np.log2(5000) / 32, 0.5, 0.0]
    # n = 8192: the sample takes every other key (i * n / 4096 = 2i)
    keys = np.zeros(8192, dtype=np.uint64)
    keys[1::2] = 0xFF
    f = M.features(keys, has_values=True)
    assert f[0] == 1.0 and f[0xFF] == 0.0
    assert f[M.P * M.R:].tolist() == [13 / 32, 1.0, 1.0]
    # fewer than 4096 keys: all of them; bit range [4, 12) -> one place of 8 bits
    keys = np.arange(16, dtype=np.uint32) << 4
    f = M.features(keys, 4, 12)
    assert np.all(f[:16] == 1 / 16) and f[:M.R].sum() == 1.0
    assert not f[M.R: M.P * M.R].any()
