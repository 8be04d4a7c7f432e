"""Pins of the FP64 surrogate-network oracle (finite differences, hand-worked Adam, BF16 rounding).

The surrogate itself is not in the paper, so its quality is parity unpinned; its
arithmetic (forward, backward, optimiser) is pinned here.
"""
import math

import numpy as np

import oracle


def _net(d_in=7, hidden=12, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = oracle.mlp_param_count(d_in, hidden)
    p = rng.standard_normal(n) * 0.3
    x = rng.standard_normal((9, d_in)) * 2.0 + 1.0
    y = rng.standard_normal((9, 2))
    mean = x.mean(axis=0)
    invstd = 1.0 / x.std(axis=0)
    return p, x, y, mean, invstd


def test_param_count():
    assert oracle.mlp_param_count(50, 256) == 79362


def test_forward_matches_numpy():
    d_in, hidden = 7, 12
    p, x, y, mean, invstd = _net(d_in, hidden)
    o = 0
    w1 = p[o:o + hidden * d_in].reshape(hidden, d_in); o += hidden * d_in
    b1 = p[o:o + hidden]; o += hidden
    w2 = p[o:o + hidden * hidden].reshape(hidden, hidden); o += hidden * hidden
    b2 = p[o:o + hidden]; o += hidden
    w3 = p[o:o + 2 * hidden].reshape(2, hidden); o += 2 * hidden
    b3 = p[o:o + 2]
    xh = (x - mean) * invstd
    h1 = np.maximum(xh @ w1.T + b1, 0)
    h2 = np.maximum(h1 @ w2.T + b2, 0)
    ref = h2 @ w3.T + b3
    np.testing.assert_allclose(oracle.mlp_forward(p, x, mean, invstd, hidden), ref, rtol=1e-12)


def test_gradient_finite_differences():
    d_in, hidden = 7, 12
    p, x, y, mean, invstd = _net(d_in, hidden)
    loss, g = oracle.mlp_gradient(p, x, y, mean, invstd, hidden)
    out = oracle.mlp_forward(p, x, mean, invstd, hidden)
    assert abs(loss - 0.5 * np.mean(np.sum((out - y) ** 2, axis=1))) < 1e-12
    h = 1e-6
    rng = np.random.Generator(np.random.PCG64(1))
    for i in rng.choice(p.size, 40, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (oracle.mlp_gradient(pp, x, y, mean, invstd, hidden)[0] -
              oracle.mlp_gradient(pm, x, y, mean, invstd, hidden)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_bf16_emulation_rounds():
    """Emulation changes results by about the BF16 unit roundoff (2^-9), no more."""
    d_in, hidden = 7, 12
    p, x, y, mean, invstd = _net(d_in, hidden)
    a = oracle.mlp_forward(p, x, mean, invstd, hidden, emulate=False)
    b = oracle.mlp_forward(p, x, mean, invstd, hidden, emulate=True)
    rel = np.linalg.norm(a - b) / np.linalg.norm(a)
    assert 1e-5 < rel < 3e-2


def test_bf16_emulated_backward_hand_worked():
    """One row through a 1 -> 1 -> 1 -> 2 network whose values need few bits, so the
    emulated BF16 roundings (8 significant bits) can be followed by hand. Each
    rounding of the backward pass (dh2, h1, w2, dh1, xh) changes a stated entry:
    dropping one, or rounding a value the GPU keeps in FP32, fails an assertion.

    Forward: xh = 3 + 2^-8 (BF16: 3); h1 = 1 * 3 + b1 = 3 + 2^-8;
    w2 = 1 + 2^-7 + 2^-11 (BF16: 1 + 2^-7); h2 = bf16(w2) bf16(h1) = (1 + 2^-7) 3;
    out = (h2, 0).
    Target y0 = h2 - e with e = 1 + 2^-7 + 2^-10, so dh2 = e (BF16: 1 + 2^-7).
    Backward: g_b3 = (e, 0), g_w3 = (e h2, 0), g_b2 = dh2 = e,
    g_w2 = bf16(dh2) bf16(h1) = (1 + 2^-7) 3,
    dh1 = bf16(dh2) bf16(w2) = (1 + 2^-7)^2 = 1 + 2^-6 + 2^-14 (exact in FP32),
    g_b1 = dh1, g_w1 = bf16(dh1) bf16(xh) = (1 + 2^-6) 3.
    """
    e = 1 + 2.0 ** -7 + 2.0 ** -10
    h2 = (1 + 2.0 ** -7) * 3
    # packed: W1 [1][1], b1 [1], W2 [1][1], b2 [1], W3 [2][1], b3 [2]
    w2 = 1 + 2.0 ** -7 + 2.0 ** -11
    params = np.array([1.0, 2.0 ** -8, w2, 0.0, 1.0, 0.0, 0.0, 0.0])
    x = np.array([[3 + 2.0 ** -8]])
    y = np.array([[h2 - e, 0.0]])
    mean, invstd = np.zeros(1), np.ones(1)
    out = oracle.mlp_forward(params, x, mean, invstd, hidden=1, emulate=True)
    np.testing.assert_array_equal(out, [[h2, 0.0]])
    loss, g = oracle.mlp_gradient(params, x, y, mean, invstd, hidden=1, emulate=True)
    assert loss == 0.5 * e * e
    dh1 = 1 + 2.0 ** -6 + 2.0 ** -14
    expect = [
        (1 + 2.0 ** -6) * 3,  # g_w1 = bf16(dh1) bf16(xh)
        dh1,                  # g_b1
        (1 + 2.0 ** -7) * 3,  # g_w2 = bf16(dh2) bf16(h1)
        e,                    # g_b2
        e * h2, 0.0,          # g_w3
        e, 0.0,               # g_b3
    ]
    np.testing.assert_array_equal(g, expect)
    # without emulation the same network follows plain double arithmetic
    _, g_plain = oracle.mlp_gradient(params, x, y, mean, invstd, hidden=1, emulate=False)
    h1 = 3 + 2.0 ** -8 + 2.0 ** -8
    assert g_plain[2] == (h1 * w2 - (h2 - e)) * h1


def test_adam_hand_worked():
    """Step 1 with m = v = 0: m = 0.1 g, v = 0.001 g^2, bias-corrected to g and g^2,
    so p moves by lr * g / (|g| + eps), i.e. lr * sign(g)."""
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    m = np.zeros(3)
    v = np.zeros(3)
    oracle.adam(p, g, m, v, 0.01, 0.9, 0.999, 1e-8, 1)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
    np.testing.assert_allclose(p, [1.0 - 0.01 * 0.3 / (0.3 + 1e-8), -2.0 + 0.01 * 4.0 / (4.0 + 1e-8),
                                   0.5], rtol=1e-15)
    # step 2 with the same gradient: bias corrections 1 - 0.81 and 1 - 0.998001
    p2 = p.copy()
    oracle.adam(p2, g, m, v, 0.01, 0.9, 0.999, 1e-8, 2)
    mh = (0.9 * 0.1 * g + 0.1 * g) / (1 - 0.9 ** 2)
    vh = (0.999 * 0.001 * g * g + 0.001 * g * g) / (1 - 0.999 ** 2)
    np.testing.assert_allclose(p2, p - 0.01 * mh / (np.sqrt(vh) + 1e-8), rtol=1e-14)
    assert math.isfinite(p2.sum())


def test_bf16_rounding_matches_torch():
    """The emulated rounding equals torch's float32 -> bfloat16 conversion (RNE)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(4))
    a = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.bf16_round(a), ref)
