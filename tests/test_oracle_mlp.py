"""Pins of the oracle's MLP (4 -> 64 -> 64 -> 4, SiLU), BF16 rounding and
Adam, no GPU.

- Back-propagation against FP64 central finite differences of the loss.
- BF16 round-to-nearest-even on values whose rounding is known by hand.
- Forward of hand-built networks with known outputs.
- Adam's first step is -lr * sign(g) (bias correction, Kingma and Ba).
"""
import math

import numpy as np

import oracle

P = oracle.MLP_NPARAM
OW1, OB1, OW2, OB2, OW3, OB3 = 0, 256, 320, 4416, 4480, 4736


def _params(seed, scale=0.3):
    r = np.random.default_rng(seed)
    return scale * r.standard_normal(P)


def test_bf16_rounding_known_values():
    e = 2.0 ** -8
    assert oracle.bf16_round(1.0 + e) == 1.0                     # tie -> even
    assert oracle.bf16_round(1.0 + 3 * e) == 1.0 + 4 * e          # tie -> even (up)
    assert oracle.bf16_round(1.0 + 1.5 * e) == 1.0 + 2 * e        # above the tie
    assert oracle.bf16_round(-(1.0 + 0.9 * e)) == -1.0
    assert oracle.bf16_round(3.0) == 3.0
    assert oracle.bf16_round(1.0 / 3.0) == 0.333984375            # 0x3EAB
    assert math.isnan(oracle.bf16_round(float("nan")))


def test_forward_hand_built():
    p = np.zeros(P)
    p[OB3:OB3 + 4] = [1.5, -2.0, 0.25, 0.0]
    x = np.random.default_rng(0).standard_normal((5, 4))
    assert np.array_equal(oracle.mlp_forward(p, x), np.tile(p[OB3:OB3 + 4], (5, 1)))
    # y0 = sum_j silu(x0) over one hidden unit chain: W1[0,0]=1, W2[0,0]=1, W3[0,0]=1
    p = np.zeros(P)
    p[OW1 + 0] = 1.0
    p[OW2 + 0] = 1.0
    p[OW3 + 0] = 1.0
    silu = lambda z: z / (1 + math.exp(-z))
    y = oracle.mlp_forward(p, x)
    for b in range(5):
        assert abs(y[b, 0] - silu(silu(x[b, 0]))) < 1e-15
        assert y[b, 1] == y[b, 2] == y[b, 3] == 0.0


def test_gradient_matches_finite_differences():
    p = _params(1)
    r = np.random.default_rng(2)
    x = r.standard_normal((7, 4))
    t = r.standard_normal((7, 4))
    loss, g = oracle.mlp_loss_grad(p, x, t)
    idx = list(range(0, 8)) + list(range(OB1, OB1 + 4)) + list(range(OW2, OW2 + 6)) + \
        list(range(OB2 + 10, OB2 + 14)) + list(range(OW3 + 60, OW3 + 70)) + list(range(OB3, OB3 + 4))
    idx += list(r.integers(0, P, 40))
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = oracle.mlp_loss_grad(pp, x, t)
        lm, _ = oracle.mlp_loss_grad(pm, x, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), i


def test_bf16_mode_is_close_to_fp64_mode():
    p = _params(3, 0.2)
    r = np.random.default_rng(4)
    x = r.standard_normal((64, 4))
    t = r.standard_normal((64, 4))
    y64 = oracle.mlp_forward(p, x)
    y16 = oracle.mlp_forward(p, x, bf16=True)
    assert np.abs(y16 - y64).max() < 0.05 * np.abs(y64).max()
    l64, g64 = oracle.mlp_loss_grad(p, x, t)
    l16, g16 = oracle.mlp_loss_grad(p, x, t, bf16=True)
    assert abs(l16 - l64) < 0.02 * l64
    assert np.abs(g16 - g64).max() < 0.05 * np.abs(g64).max()


def test_adam_first_step_is_sign():
    r = np.random.default_rng(5)
    g = r.standard_normal(P)
    p = np.zeros(P)
    m = np.zeros(P)
    v = np.zeros(P)
    oracle.adam_step(p, m, v, g, 1, lr=1e-3)
    want = -1e-3 * g / (np.abs(g) + 1e-8)   # = -lr sign(g) up to eps
    assert np.allclose(p, want, rtol=1e-12, atol=0)
    # a constant gradient keeps the step at that value (bias correction)
    for t in range(2, 6):
        q = p.copy()
        oracle.adam_step(p, m, v, g, t, lr=1e-3)
        assert np.allclose(p - q, want, rtol=1e-9, atol=0)
