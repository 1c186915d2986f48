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


def test_elbm_alpha_constant_entropy_and_lbgk_limit():
    """S(f + alpha (f* - f)) = S(f) at the returned alpha; alpha -> 2 (the
    LBGK mirror) as f -> f*."""
    _, _, w = oracle.velocities(9)
    r = np.random.default_rng(6)
    for scale in (1e-1, 1e-2, 1e-3):
        for _ in range(10):
            fs = oracle.qe_entropic_mm(9, r.uniform(0.5, 1.5), r.uniform(-0.1, 0.1), r.uniform(-0.1, 0.1))
            d = scale * fs * r.uniform(-1, 1, 9)
            # keep mass and momentum (the entropic QE of f is then fs)
            vx, vy, _ = oracle.velocities(9)
            A = np.stack([np.ones(9), vx, vy]).astype(float)
            d -= A.T @ np.linalg.solve(A @ A.T, A @ d)
            f = fs + d
            a = oracle.elbm_alpha(f, fs)
            S0 = _perfect_entropy(f, w)
            S1 = _perfect_entropy(f + a * (fs - f), w)
            assert abs(S1 - S0) < 1e-12
            assert abs(a - 2.0) < 5 * scale
