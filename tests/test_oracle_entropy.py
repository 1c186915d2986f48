"""Pins of the oracle's nonequilibrium entropy Delta S (Sec. 3.3) and of the
ELBM entropic involution parameter (Sec. 3.2, Sec. 4.1), no GPU."""
import decimal
import math

import numpy as np
import pytest

import oracle


def _perfect_entropy(f, w):
    return -sum(fi * math.log(fi / wi) for fi, wi in zip(f, w) if fi > 0)


def test_zero_at_equilibrium_and_nonnegative():
    r = np.random.default_rng(1)
    for _ in range(200):
        rho, u1, u2 = r.uniform(0.5, 1.5), r.uniform(-0.1, 0.1), r.uniform(-0.1, 0.1)
        fs = oracle.qe_poly(9, rho, u1, u2)
        assert oracle.delta_S(fs, fs) == 0.0
        f = fs * (1 + 0.05 * r.standard_normal(9))
        assert oracle.delta_S(f, fs) > 0.0


def test_equals_entropy_difference_for_entropic_quasiequilibrium():
    """For the entropic f*_M with m(f) = m(f*), Delta S = S(f*) - S(f) with
    the perfect entropy S = -sum f ln(f/W) (the definition in Sec. 3.3)."""
    vx, vy, w = oracle.velocities(9)
    rows = np.stack([np.ones(9), vx, vy, vx * vx + vy * vy]).astype(float)
    r = np.random.default_rng(2)
    for _ in range(100):
        f = oracle.qe_poly(9, r.uniform(0.5, 1.5), r.uniform(-0.1, 0.1), r.uniform(-0.1, 0.1))
        f = f * (1 + 0.1 * r.uniform(-1, 1, 9))
        M = rows @ f
        mu, it, _ = oracle.fstar_newton(M)
        fs = oracle.fstar_from_mu(mu)
        want = _perfect_entropy(fs, w) - _perfect_entropy(f, w)
        # the identity holds up to (lambda + e_0) . (m(f*) - M), lambda the
        # multipliers of ln(f*/W) (the -f + f* terms give the e_0 part), plus
        # ~1e-15 from the FP64 difference of two O(1) entropies
        lam = mu - np.array([math.log(4 / 9) - 1, 0, 0, -math.log(4)])
        bound = float(np.abs(lam) @ np.abs(rows @ fs - M)) + 1e-14
        assert abs(oracle.delta_S(f, fs) - want) <= bound


def test_matches_kullback_form_when_masses_agree():
    r = np.random.default_rng(3)
    for _ in range(100):
        fs = oracle.qe_poly(9, r.uniform(0.5, 1.5), r.uniform(-0.1, 0.1), r.uniform(-0.1, 0.1))
        d = r.uniform(-1, 1, 9) * 0.05 * fs
        d -= d.mean()
        f = fs + d
        kull = float(np.sum(f * np.log(f / fs)))
        assert abs(oracle.delta_S(f, fs) - kull) < 1e-14


def _decimal_dS(f, fs):
    decimal.getcontext().prec = 50
    acc = decimal.Decimal(0)
    for a, b in zip(f, fs):
        a, b = decimal.Decimal(float(a)), decimal.Decimal(float(b))
        acc += a * (a / b).ln() - a + b
    return float(acc)


def test_high_precision_value():
    """50-digit decimal evaluation of the same sum, down to Delta S ~ 1e-14.
    The long-double direct sum carries an absolute error of order
    eps_ld * sum(f) (eps_ld ~ 1.1e-19) from the cancellation of
    f ln(f/f*) against f - f*, plus the final rounding to FP64."""
    r = np.random.default_rng(4)
    for scale in (1e-1, 1e-3, 1e-5, 1e-7):
        for _ in range(20):
            fs = oracle.qe_poly(9, r.uniform(0.5, 1.5), r.uniform(-0.1, 0.1), r.uniform(-0.1, 0.1))
            f = fs * (1 + scale * r.uniform(-1, 1, 9))
            want = _decimal_dS(f, fs)
            assert abs(oracle.delta_S(f, fs) - want) <= 2.3e-16 * want + 1e-18 * f.sum()


def test_quadratic_limit():
    r = np.random.default_rng(5)
    fs = oracle.qe_poly(9, 1.0, 0.03, -0.02)
    for _ in range(20):
        d = 1e-5 * fs * r.uniform(-1, 1, 9)
        quad = float(np.sum(d * d / (2 * fs)))
        assert abs(oracle.delta_S(fs + d, fs) - quad) < 1e-4 * quad


def test_invalid_sites():
    fs = oracle.qe_poly(3, 1.0, 0.0)
    assert oracle.delta_S(np.array([0.7, -1e-3, 0.3]), fs) == math.inf
    assert oracle.delta_S(fs, np.array([0.7, 0.0, 0.3])) == math.inf
    f = np.array([0.0, 1 / 6, 1 / 6])
    # a zero population contributes its limit f*_i
    want = 0.0 + 2 / 3 + 0.0 + 0.0
    assert abs(oracle.delta_S(f, fs) - want) < 1e-15


def _mm_perturbed(r, scale, Q=9):
    """An entropic mass-momentum quasiequilibrium and a state with its mass
    and momentum (so that f* is the quasiequilibrium of f)."""
    vx, vy, w = oracle.velocities(Q)
    u2 = r.uniform(-0.1, 0.1) if Q == 9 else 0.0
    fs = oracle.qe_entropic_mm(Q, r.uniform(0.5, 1.5), r.uniform(-0.1, 0.1), u2)
    d = scale * fs * r.uniform(-1, 1, Q)
    A = np.stack([np.ones(Q), vx, vy]).astype(float)[: 2 if Q == 3 else 3]
    d -= A.T @ np.linalg.solve(A @ A.T, A @ d)
    return fs + d, fs, w


def test_elbm_entropy_function_equals_entropy_difference():
    """The cancellation-free H(a) equals S(f + a(f* - f)) - S(f) (50-digit
    decimal) where that difference is well conditioned."""
    decimal.getcontext().prec = 60
    D = decimal.Decimal
    r = np.random.default_rng(8)
    for Q in (3, 9):
        for _ in range(20):
            f, fs, w = _mm_perturbed(r, 0.1, Q)
            for a in (0.5, 1.0, 1.7, 2.0, 2.3):
                if not (f + a * (fs - f) > 0).all():
                    continue
                Df, Dfs, Dw, Da = [D(float(v)) for v in f], [D(float(v)) for v in fs], [D(float(v)) for v in w], D(a)
                g = [x + Da * (y - x) for x, y in zip(Df, Dfs)]
                S = lambda h: -sum(hi * (hi / wi).ln() for hi, wi in zip(h, Dw))
                want = float(S(g) - S(Df))
                # the exact rewrite drops sum (f* - f)(1 + ln(f*/W)), which is
                # zero up to the FP64 rounding of f*
                corr = float(sum((y - x) * (D(1) + (y / wi).ln()) for x, y, wi in zip(Df, Dfs, Dw)))
                assert abs(oracle.elbm_H(f, fs, a) - (want + a * corr)) <= 1e-14 * max(abs(want), 1e-6)


def test_elbm_alpha_constant_entropy_and_lbgk_limit():
    """H(alpha) = 0 at the returned alpha (the root is bracketed to 1e-15);
    alpha -> 2 (the LBGK mirror) as f -> f*."""
    r = np.random.default_rng(6)
    for scale in (1e-1, 1e-2, 1e-3, 1e-5, 1e-7):
        for _ in range(10):
            f, fs, w = _mm_perturbed(r, scale)
            a = oracle.elbm_alpha(f, fs)
            assert oracle.elbm_H(f, fs, a - 1e-14) > 0 > oracle.elbm_H(f, fs, a + 1e-14)
            assert abs(a - 2.0) < 5 * scale
