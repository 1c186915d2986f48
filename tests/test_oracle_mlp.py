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


# ---------------------------------------------------------------------------
# Inputs and outputs of the warm-start network (or_mlp_features,
# or_mlp_targets, or_mlp_unnormalise), pinned without the functions' own
# formulas: hand-computed values, the density scaling of f*_M, and the
# isothermal closed form of Sec. 4.2 reached by the independent scalar route.
# ---------------------------------------------------------------------------
IDENT = [0.0] * 4 + [1.0] * 4 + [0.0] * 4 + [1.0] * 4


def _M(rho, u1, u2, e):
    return np.array([[rho], [rho * u1], [rho * u2], [rho * e]], np.float64)


def test_features_hand_computed():
    # rho = 2, rho u = (0.25, -0.125), 2E = 1.5: u = (0.125, -0.0625),
    # 2E/rho = 0.75, |u|^2 = 0.01953125 (all exact in binary)
    M = np.array([[2.0], [0.25], [-0.125], [1.5]])
    X = oracle.mlp_features(M, IDENT)
    assert X.shape == (1, 4)
    assert X[0].tolist() == [0.125, -0.0625, 0.75, 0.01953125]
    # shifts and scales act per feature: (v - shift) * scale
    nm = [0.125, 0.0, 0.5, 0.0, 8.0, -16.0, 4.0, 256.0] + [0.0] * 4 + [1.0] * 4
    X = oracle.mlp_features(M, nm)
    assert X[0].tolist() == [0.0, 1.0, 1.0, 5.0]
    # rounded to FP32 as the network receives them: 0.1 is not a float
    X = oracle.mlp_features(np.array([[1.0], [0.1], [0.0], [0.7]]), IDENT)
    assert X[0, 0] == float(np.float32(0.1)) and X[0, 0] != 0.1


def test_features_density_scaling_and_layout():
    r = np.random.default_rng(7)
    n = 9
    rho = r.uniform(0.5, 1.5, n)
    u1, u2 = r.uniform(-0.1, 0.1, (2, n))
    e = 2.0 / 3.0 + u1 ** 2 + u2 ** 2
    M = np.stack([rho, rho * u1, rho * u2, rho * e])
    X = oracle.mlp_features(M, IDENT)
    for lam in (0.25, 3.0):
        assert np.abs(oracle.mlp_features(lam * M, IDENT) - X).max() <= 1e-7 * np.abs(X).max()
    # sample-major output, component-major input: sample s reads column s
    for s in range(n):
        xs = oracle.mlp_features(M[:, s:s + 1], IDENT)[0]
        assert np.array_equal(xs, X[s])
    assert np.allclose(X[:, 0], u1, rtol=1e-7, atol=0) and np.allclose(X[:, 3], u1 ** 2 + u2 ** 2, rtol=1e-6)


def _closed_form_targets(u1, u2):
    # Sec. 4.2's product formula: f*_i = rho W_i prod_j (2 - s_j) B_j^{v_ij},
    # s_j = sqrt(1 + 3 u_j^2), B_j = (2 u_j + s_j) / (1 - u_j); with
    # W = (4/9, 1/9, 1/36) = (4/9) (1/4)^{|v|^2}, ln f*_i is linear in
    # (1, vx, vy, |v|^2) with coefficients (ln(4 rho/9) + ln((2-sx)(2-sy)),
    # ln Bx, ln By, -ln 4)
    sx, sy = math.sqrt(1 + 3 * u1 * u1), math.sqrt(1 + 3 * u2 * u2)
    return [math.log(4.0 / 9.0) + math.log((2 - sx) * (2 - sy)), math.log((2 * u1 + sx) / (1 - u1)),
            math.log((2 * u2 + sy) / (1 - u2)), -math.log(4.0)]


def test_targets_isothermal_closed_form():
    for rho, u1, u2 in ((1.0, 0.0, 0.0), (0.7, 0.05, -0.08), (1.4, -0.09, 0.02)):
        e = -2.0 / 3.0 + (2.0 / 3.0) * (math.sqrt(1 + 3 * u1 * u1) + math.sqrt(1 + 3 * u2 * u2))
        M = _M(rho, u1, u2, e)
        mu = oracle.fstar_scalar(M[:, 0]).reshape(4, 1)
        T = oracle.mlp_targets(M, mu, IDENT)[0]
        want = _closed_form_targets(u1, u2)
        assert np.abs(T - want).max() < 1e-12, (T, want)
        # normalisation: (v - shift) * scale with the output constants (held
        # in FP32, like the network's)
        s0 = float(np.float32(want[0]))
        nm = [0.0] * 8 + [s0, 0.0, 1.0, -1.0] + [2.0, 4.0, 0.5, 8.0]
        Tn = oracle.mlp_targets(M, mu, nm)[0]
        ref = [(want[0] - s0) * 2.0, want[1] * 4.0, (want[2] - 1.0) * 0.5, (want[3] + 1.0) * 8.0]
        assert np.abs(Tn - ref).max() < 1e-11


def test_targets_density_scaling():
    # M -> lambda M: mu0 -> mu0 + ln lambda, mu1..3 unchanged, so the targets
    # (mu0 - ln rho, mu1, mu2, mu3) do not change (each mu from its own solve)
    M = _M(0.9, 0.06, -0.03, 0.70)
    mu, it, res = oracle.fstar_newton(M[:, 0], 1e-14)
    assert it >= 0
    T = oracle.mlp_targets(M, mu.reshape(4, 1), IDENT)[0]
    for lam in (0.3, 2.5):
        mul, itl, _ = oracle.fstar_newton(lam * M[:, 0], 1e-14)
        assert itl >= 0
        Tl = oracle.mlp_targets(lam * M, mul.reshape(4, 1), IDENT)[0]
        assert np.abs(Tl - T).max() < 1e-12


def test_warm_start_constant_network_and_unnormalise():
    # a network with zero weights outputs its last bias b3 for every input:
    # the warm start is then b3 / out_scale + out_shift, component-major
    p = np.zeros(P)
    p[OB3:OB3 + 4] = [1.0, -2.0, 0.5, 4.0]
    nm = [0.0] * 4 + [1.0] * 4 + [-0.5, 0.25, 2.0, -1.0] + [2.0, 4.0, 0.5, 8.0]
    M = np.stack([np.full(3, 1.2), [0.01, 0.02, 0.03], [0.0, -0.01, 0.02], np.full(3, 0.8)])
    W = oracle.mlp_warm_start(p, nm, M)
    assert W.shape == (4, 3)
    want = [1.0 / 2.0 - 0.5, -2.0 / 4.0 + 0.25, 0.5 / 0.5 + 2.0, 4.0 / 8.0 - 1.0]
    for s in range(3):
        assert W[:, s].tolist() == want
    # unnormalise inverts the target normalisation exactly (up to rounding)
    mu = np.array([[-0.9], [0.1], [-0.2], [-1.4]])
    Mt = _M(1.3, 0.0, 0.0, 0.6)
    T = oracle.mlp_targets(Mt, mu, nm)
    back = oracle.mlp_unnormalise(T, nm)[:, 0]
    assert np.abs(back - [mu[0, 0] - math.log(1.3), 0.1, -0.2, -1.4]).max() < 1e-15


def test_warm_start_depends_on_the_normalised_features():
    # one hidden chain reading feature 2 (2E/rho) only: moments with the same
    # 2E/rho give the same start whatever their density and velocity, and a
    # different 2E/rho gives a different start
    p = np.zeros(P)
    p[OW1 + 2] = 1.0      # W1[0][2]
    p[OW2 + 0] = 1.0      # W2[0][0]
    p[OW3 + 0] = 1.0      # W3[0][0]
    nm = [0.0, 0.0, 0.6, 0.0] + [1.0, 1.0, 10.0, 1.0] + [0.0] * 4 + [1.0] * 4
    a = oracle.mlp_warm_start(p, nm, _M(1.0, 0.01, 0.02, 0.7))
    b = oracle.mlp_warm_start(p, nm, _M(1.4, -0.05, 0.03, 0.7))
    c = oracle.mlp_warm_start(p, nm, _M(1.0, 0.01, 0.02, 0.75))
    silu = lambda z: z / (1 + math.exp(-z))
    assert a[0, 0] == b[0, 0]
    assert abs(a[0, 0] - silu(oracle.bf16_round(silu(1.0)))) < 1e-2   # x2 = (0.7 - 0.6) * 10 = 1
    assert abs(c[0, 0] - silu(oracle.bf16_round(silu(1.5)))) < 1e-2
    assert a[1:, 0].tolist() == [0.0, 0.0, 0.0]
