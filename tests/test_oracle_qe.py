"""Pins of the oracle's lattice tables and quasiequilibria against what the
paper and the mathematics fix (no GPU).

- Velocity numbering and weights: fixtures typed from Sec. 4.1 / Sec. 4.2.
- Polynomial quasiequilibria: exact mass, momentum and second moments; the
  D2Q9 polynomial's u2 = 0 marginal is Sec. 4.1's D1Q3 formula.
- Entropic quasiequilibria: constraint satisfaction plus optimality (the
  entropy decreases along every direction that keeps the constraints), and
  the KKT structure ln f* in the span of the moment rows (Sec. 3.3).
- f*_M: two independent routes (4x4 Newton, scalar reduction) agree; the
  isothermal special case reproduces the closed form of Sec. 4.2.
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows = []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append([int(t) for t in line.split()])
    return np.array(rows)


def test_d2q9_table_matches_paper_numbering():
    g = _read("d2q9_lattice.txt")
    vx, vy, w = oracle.velocities(9)
    assert np.array_equal(vx, g[:, 1]) and np.array_equal(vy, g[:, 2])
    assert np.allclose(w, g[:, 3] / g[:, 4], rtol=0, atol=1e-16)


def test_d1q3_table_matches_paper():
    g = _read("d1q3_lattice.txt")
    vx, vy, w = oracle.velocities(3)
    assert np.array_equal(vx, g[:, 1]) and not vy.any()
    assert np.allclose(w, g[:, 2] / g[:, 3], rtol=0, atol=1e-16)


def test_weights_isotropy_and_tensor_product():
    vx, vy, w = oracle.velocities(9)
    v1, _, w1 = oracle.velocities(3)
    assert abs(w.sum() - 1) < 1e-15
    assert abs((w * vx * vx).sum() - 1 / 3) < 1e-15 and abs((w * vy * vy).sum() - 1 / 3) < 1e-15
    assert abs((w * vx * vy).sum()) < 1e-15
    # D2Q9 weights are products of the D1Q3 weights of each component
    wd = {int(v): float(ww) for v, ww in zip(v1, w1)}
    for i in range(9):
        assert abs(w[i] - wd[int(vx[i])] * wd[int(vy[i])]) < 1e-16


def _rand_states(n, seed, umax=0.15):
    r = np.random.default_rng(seed)
    return [(float(r.uniform(0.3, 2.0)), float(r.uniform(-umax, umax)), float(r.uniform(-umax, umax)))
            for _ in range(n)]


@pytest.mark.parametrize("Q", [3, 9])
def test_poly_qe_moments(Q):
    vx, vy, _ = oracle.velocities(Q)
    for rho, u1, u2 in _rand_states(50, 1):
        if Q == 3:
            u2 = 0.0
        fs = oracle.qe_poly(Q, rho, u1, u2)
        assert abs(fs.sum() - rho) < 1e-14
        assert abs((vx * fs).sum() - rho * u1) < 1e-14
        assert abs((vy * fs).sum() - rho * u2) < 1e-14
        # second moments: rho (delta_ab / 3 + u_a u_b)
        assert abs((vx * vx * fs).sum() - rho * (1 / 3 + u1 * u1)) < 1e-14
        if Q == 9:
            assert abs((vy * vy * fs).sum() - rho * (1 / 3 + u2 * u2)) < 1e-14
            assert abs((vx * vy * fs).sum() - rho * u1 * u2) < 1e-14


def test_poly_d2q9_marginal_is_printed_d1q3():
    """Summing the D2Q9 polynomial over v_y at u2 = 0 gives Sec. 4.1's D1Q3."""
    vx, vy, _ = oracle.velocities(9)
    v1, _, _ = oracle.velocities(3)
    for rho, u1, _ in _rand_states(20, 2):
        f9 = oracle.qe_poly(9, rho, u1, 0.0)
        f3 = oracle.qe_poly(3, rho, u1)
        for j, v in enumerate(v1):
            assert abs(f9[vx == v].sum() - f3[j]) < 1e-15


def _entropy(f, w):
    return -np.sum(f * np.log(f / w))


def _null_space(rows):
    u, s, vt = np.linalg.svd(rows)
    rank = int((s > 1e-12).sum())
    return vt[rank:]


@pytest.mark.parametrize("Q", [3, 9])
def test_entropic_mm_is_constrained_entropy_maximum(Q):
    vx, vy, w = oracle.velocities(Q)
    rows = np.stack([np.ones(Q), vx, vy])[: 2 if Q == 3 else 3].astype(float)
    N = _null_space(rows)
    r = np.random.default_rng(3)
    for rho, u1, u2 in _rand_states(30, 3, umax=0.3):
        if Q == 3:
            u2 = 0.0
        fs = oracle.qe_entropic_mm(Q, rho, u1, u2)
        assert (fs > 0).all()
        assert abs(fs.sum() - rho) < 1e-14
        assert abs((vx * fs).sum() - rho * u1) < 1e-14  # +rho u: the corrected D1Q3 pair
        assert abs((vy * fs).sum() - rho * u2) < 1e-14
        # ln(f*/W) in the span of the constraint rows (Lagrange form, Sec. 3.3)
        lw = np.log(fs / w)
        coef, *_ = np.linalg.lstsq(rows.T, lw, rcond=None)
        assert np.abs(rows.T @ coef - lw).max() < 1e-12
        S0 = _entropy(fs, w)
        for _ in range(5):
            d = r.standard_normal(N.shape[0]) @ N
            d *= 1e-3 * fs.min() / np.abs(d).max()
            assert _entropy(fs + d, w) < S0
            assert _entropy(fs - d, w) < S0


def test_d1q3_entropic_as_printed_has_reversed_momentum():
    """The printed f2 (left-moving) and f3 (right-moving) of Sec. 4.1 carry
    momentum -rho u; the oracle's exchanged pair carries +rho u."""
    rho, u = 1.0, 0.1
    s = math.sqrt(1 + 3 * u * u)
    f2_printed = rho / 6 * ((3 * u - 1) + 2 * s)
    f3_printed = -rho / 6 * ((3 * u + 1) - 2 * s)
    assert abs((f3_printed - f2_printed) - (-rho * u)) < 1e-15
    fs = oracle.qe_entropic_mm(3, rho, u)
    assert abs((fs[2] - fs[1]) - rho * u) < 1e-15


def test_d2q9_entropic_mm_factorises_into_d1q3():
    """Sec. 4.2's D2Q9 formula is the product of 1-D factors whose x-marginal
    at u2 = 0 is the (corrected) D1Q3 entropic quasiequilibrium."""
    vx, vy, _ = oracle.velocities(9)
    v1, _, _ = oracle.velocities(3)
    for rho, u1, _ in _rand_states(20, 4, umax=0.3):
        f9 = oracle.qe_entropic_mm(9, rho, u1, 0.0)
        f3 = oracle.qe_entropic_mm(3, rho, u1)
        for j, v in enumerate(v1):
            assert abs(f9[vx == v].sum() - f3[j]) < 1e-15


# ---------------------------------------------------------------------------
# f*_M with the energy row
# ---------------------------------------------------------------------------

def _moment_rows():
    vx, vy, _ = oracle.velocities(9)
    return np.stack([np.ones(9), vx, vy, vx * vx + vy * vy]).astype(float)


def _random_M(n, seed, umax=0.1, band=0.05):
    import workloads
    return workloads.random_moments(n, seed, umax=umax, energy_band=band).T


def test_fstar_newton_residual_and_optimality():
    rows = _moment_rows()
    N = _null_space(rows)
    _, _, w = oracle.velocities(9)
    r = np.random.default_rng(5)
    for M in _random_M(200, 11, umax=0.3, band=0.3):
        mu, it, res = oracle.fstar_newton(M)
        assert it >= 0 and res <= 1e-13
        fs = oracle.fstar_from_mu(mu)
        assert np.abs(rows @ fs - M).max() / M[0] <= 1e-13
        S0 = _entropy(fs, w)
        for _ in range(3):
            d = r.standard_normal(N.shape[0]) @ N
            d *= 1e-3 * fs.min() / np.abs(d).max()
            assert _entropy(fs + d, w) < S0 and _entropy(fs - d, w) < S0


def test_fstar_two_routes_agree():
    for M in _random_M(300, 12, umax=0.3, band=0.3):
        mu_n, it, _ = oracle.fstar_newton(M)
        mu_s = oracle.fstar_scalar(M)
        assert it >= 0 and mu_s is not None
        fn, fsc = oracle.fstar_from_mu(mu_n), oracle.fstar_from_mu(mu_s)
        assert np.abs(fn - fsc).max() / M[0] < 1e-12


def test_fstar_isothermal_energy_gives_closed_form():
    """At 2E/rho = -2/3 + (2/3)(sqrt(1+3u1^2) + sqrt(1+3u2^2)) the energy
    constraint is inactive: f*_M equals Sec. 4.2's mass-momentum formula."""
    rows = _moment_rows()
    for rho, u1, u2 in _rand_states(50, 6, umax=0.3):
        cf = oracle.qe_entropic_mm(9, rho, u1, u2)
        M = rows @ cf
        e_iso = -2 / 3 + 2 / 3 * (math.sqrt(1 + 3 * u1 * u1) + math.sqrt(1 + 3 * u2 * u2))
        assert abs(M[3] / rho - e_iso) < 1e-14
        mu, it, _ = oracle.fstar_newton(M)
        assert it >= 0
        assert np.abs(oracle.fstar_from_mu(mu) - cf).max() / rho < 1e-13
        assert abs(mu[3] - math.log(0.25)) < 1e-12  # Z = 1/4


def test_fstar_density_scaling():
    for M in _random_M(30, 13):
        mu1, _, _ = oracle.fstar_newton(M)
        mu2, _, _ = oracle.fstar_newton(3.7 * M)
        assert abs(mu2[0] - mu1[0] - math.log(3.7)) < 1e-12
        assert np.abs(mu2[1:] - mu1[1:]).max() < 1e-12


def test_fstar_infeasible_is_flagged():
    assert not oracle.fstar_feasible([1.0, 0.3, 0.2, 0.49])   # 2E/rho below |u1|+|u2|
    assert not oracle.fstar_feasible([1.0, 0.0, 0.0, 2.0])    # at the upper bound
    assert not oracle.fstar_feasible([0.0, 0.0, 0.0, 0.5])
    mu, it, _ = oracle.fstar_newton([1.0, 0.3, 0.2, 0.49])
    assert it == -1
    assert oracle.fstar_feasible([1.0, 0.3, 0.2, 0.51])
    mu, it, res = oracle.fstar_newton([1.0, 0.3, 0.2, 0.51], max_iter=200)
    assert it >= 0 and res < 1e-13


def test_fstar_polish_reaches_round_off():
    """One more Newton update from a 1e-13 residual carries f*_M to FP64
    round-off: the residual drops to a few ulps and f* agrees with the
    independent long-double scalar route (Sec. 2 argmax) to ~1e-15."""
    worst_r, worst_f = 0.0, 0.0
    for M in _random_M(300, 14, umax=0.3, band=0.3):
        mu, it, res = oracle.fstar_newton(M, 1e-13)
        assert it >= 0
        mp, rp = oracle.fstar_polish(M, mu)
        assert rp <= res
        fsc = oracle.fstar_from_mu(oracle.fstar_scalar(M))
        worst_r = max(worst_r, rp)
        worst_f = max(worst_f, np.abs(oracle.fstar_from_mu(mp) - fsc).max() / M[0])
    assert worst_r < 2e-15 and worst_f < 2e-15, (worst_r, worst_f)


def test_fstar_in_step_is_polished():
    """Inside the time step f*_M is the polished solve: with delta = 0 and
    k = N every site is returned to f*_M, and free flight on the periodic
    lattice carries f*_i(x) to x + v_i; un-rolled, every site matches the
    scalar route to ~1e-15."""
    nx, ny = 9, 5
    cfg = oracle.make_cfg(Q=9, qe=oracle.QE_ENTROPIC_M, nx=nx, ny=ny, nu=1e-3, delta=0.0, k=nx * ny)
    M = _random_M(nx * ny, 15, umax=0.2, band=0.2)
    f = np.zeros((9, ny, nx))
    for s in range(nx * ny):
        f[:, s // nx, s % nx] = oracle.fstar_from_mu(oracle.fstar_scalar(M[s])) * (1 + 0.01 * np.sin(np.arange(9) + s))
    o = oracle.step(cfg, f)
    assert o["n_selected"] == nx * ny
    vx, vy, _ = oracle.velocities(9)
    back = np.stack([np.roll(np.roll(o["f"][i], -vy[i], axis=0), -vx[i], axis=1) for i in range(9)])
    rows = _moment_rows()
    for s in range(nx * ny):
        g = f[:, s // nx, s % nx]
        want = oracle.fstar_from_mu(oracle.fstar_scalar(rows @ g))
        got = back[:, s // nx, s % nx]
        assert np.abs(got - want).max() / g.sum() < 2e-15, s
