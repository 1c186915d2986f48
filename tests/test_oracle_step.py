"""Pins of the oracle's whole time step (Sec. 3.2, Sec. 4.1, Sec. 4.2), no GPU.

- Free flight (Sec. 3) is an exact permutation of each population plane and
  conserves the perfect entropy; checked with beta = 0 (nu = inf) against
  numpy.roll.
- Collision conserves mass and momentum.
- delta = inf and k = 0 both reduce eq. (ESLB) to eq. (lbgkLB).
- beta = 1/2 is the Ehrenfests' chain: the entropy never decreases (Sec. 3).
- Shear-wave decay rate pins beta(nu) = 1/(1 + 6 nu) and the sign of the
  collision (textbook LBGK: nu = (1/3)(1/(2 beta) - 1/2)).
- D2Q9 with y-uniform fields reduces to D1Q3 (tensor structure).
- Selection: brute force over the oracle's own Delta S, with forced ties and
  the "fewer than k: all of them" rule (Sec. 3.2).
- Boundary rules: a uniform free stream is an exact steady state of the
  inlet / zero-gradient / free-slip channel; closed boxes conserve mass.
- Shock tube (Sec. 4.1): Ehrenfests' steps reduce post-shock oscillation.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

INF = float("inf")


def _near_eq_state(cfg, seed, amp=0.05, umax=0.05):
    r = np.random.default_rng(seed)
    ny, nx = cfg.ny, cfg.nx
    rho = 1 + 0.1 * r.uniform(-1, 1, (ny, nx))
    u = umax * r.uniform(-1, 1, (2, ny, nx))
    f = oracle.init(cfg, rho, u)
    f *= 1 + amp * r.uniform(-1, 1, f.shape)
    return f


def test_free_flight_is_a_permutation():
    cfg = oracle.make_cfg(Q=9, nx=13, ny=7, nu=INF)
    f = _near_eq_state(cfg, 1)
    g = oracle.step(cfg, f)["f"]
    vx, vy, w = oracle.velocities(9)
    for i in range(9):
        assert np.array_equal(g[i], np.roll(np.roll(f[i], vy[i], axis=0), vx[i], axis=1))
    S = lambda h: -np.sum(h * np.log(h / w[:, None, None]))
    assert abs(S(g) - S(f)) < 1e-12 * abs(S(f))


@pytest.mark.parametrize("qe", [oracle.QE_POLY, oracle.QE_ENTROPIC_MM, oracle.QE_ENTROPIC_M])
def test_collision_conserves(qe):
    cfg = oracle.make_cfg(Q=9, qe=qe, nx=11, ny=6, nu=1e-3, delta=1e-4, k=5)
    f = _near_eq_state(cfg, 2)
    out = oracle.step(cfg, f)
    vx, vy, _ = oracle.velocities(9)
    for row in (np.ones(9), vx, vy) + ((vx * vx + vy * vy,) if qe == oracle.QE_ENTROPIC_M else ()):
        a = np.tensordot(row, f, 1).sum()
        b = np.tensordot(row, out["f"], 1).sum()
        assert abs(a - b) < 1e-12 * f.sum()
    assert out["n_selected"] == min(5, out["n_above"]) and out["n_above"] > 0


def test_delta_inf_equals_k0():
    f_cfg = dict(Q=9, nx=10, ny=5, nu=1e-4)
    a = oracle.make_cfg(delta=INF, k=8, **f_cfg)
    b = oracle.make_cfg(delta=1e-6, k=0, **f_cfg)
    f = _near_eq_state(a, 3)
    ra, rb = oracle.step(a, f), oracle.step(b, f)
    assert np.array_equal(ra["f"], rb["f"])
    assert ra["n_selected"] == 0 and rb["n_selected"] == 0 and rb["n_above"] > 0


def test_half_beta_is_ehrenfest_chain():
    """beta = 1/2 (nu = 1/6): every site goes to f* and then free-flies; the
    perfect entropy never decreases (Sec. 3)."""
    cfg = oracle.make_cfg(Q=9, qe=oracle.QE_ENTROPIC_MM, nx=12, ny=9, nu=1.0 / 6.0)
    f = _near_eq_state(cfg, 4, amp=0.2, umax=0.1)
    _, _, w = oracle.velocities(9)
    S = lambda h: -np.sum(h * np.log(h / w[:, None, None]))
    s_prev = S(f)
    for _ in range(10):
        f = oracle.step(cfg, f)["f"]
        s = S(f)
        assert s >= s_prev - 1e-13
        s_prev = s


def test_shear_wave_decay_pins_viscosity():
    nu = 0.02
    ny, nx, U = 64, 2, 1e-4
    cfg = oracle.make_cfg(Q=9, nx=nx, ny=ny, nu=nu)
    y = np.arange(ny)
    u = np.zeros((2, ny, nx))
    u[0] = (U * np.sin(2 * math.pi * y / ny))[:, None]
    f = oracle.init(cfg, np.ones((ny, nx)), u)
    vx, vy, _ = oracle.velocities(9)

    def amp(h):
        ux = np.tensordot(vx, h, 1)[:, 0] / h.sum(0)[:, 0]
        return 2 * np.mean(ux * np.sin(2 * math.pi * y / ny))

    a0 = amp(oracle.run(cfg, f, 20))
    T = 300
    a1 = amp(oracle.run(cfg, f, 20 + T))
    kk = 2 * math.pi / ny
    nu_meas = -math.log(a1 / a0) / (kk * kk * T)
    assert abs(nu_meas - nu) < 0.01 * nu


def test_d2q9_reduces_to_d1q3():
    nx = 40
    c3 = oracle.make_cfg(Q=3, nx=nx, ny=1, nu=1e-3)
    c9 = oracle.make_cfg(Q=9, nx=nx, ny=1, nu=1e-3)
    r = np.random.default_rng(5)
    rho = 1 + 0.2 * r.uniform(-1, 1, (1, nx))
    u = np.zeros((2, 1, nx))
    u[0] = 0.05 * r.uniform(-1, 1, (1, nx))
    f3 = oracle.init(c3, rho, u[:1])
    f9 = oracle.init(c9, rho, u)
    vx, _, _ = oracle.velocities(9)
    v1, _, _ = oracle.velocities(3)
    for _ in range(25):
        f3 = oracle.step(c3, f3)["f"]
        f9 = oracle.step(c9, f9)["f"]
    for j, v in enumerate(v1):
        assert np.abs(f9[vx == v].sum(0) - f3[j]).max() < 1e-14


def _brute_selection(dS, delta, k):
    cand = [(-d, s) for s, d in enumerate(dS.reshape(-1)) if d > delta]
    cand.sort()
    return [s for _, s in cand[:k]], len(cand)


@pytest.mark.parametrize("k", [0, 1, 3, 7, 50])
def test_selection_matches_brute_force(k):
    cfg = oracle.make_cfg(Q=9, nx=8, ny=6, nu=1e-3, delta=1e-5, k=k)
    f = _near_eq_state(cfg, 6, amp=0.02)
    # forced ties: copy one site's populations into three others (identical Delta S)
    f[:, 2, 5] = f[:, 0, 1]
    f[:, 4, 0] = f[:, 0, 1]
    f[:, 5, 7] = f[:, 0, 1]
    out = oracle.step(cfg, f)
    want, n_above = _brute_selection(out["dS"], cfg.delta, k)
    assert out["n_above"] == n_above and n_above > 10
    assert list(out["sel"]) == want


def test_fewer_than_k_returns_all():
    cfg = oracle.make_cfg(Q=9, nx=8, ny=6, nu=1e-3, delta=1e-5, k=1000)
    f = _near_eq_state(cfg, 7, amp=0.02)
    out = oracle.step(cfg, f)
    assert out["n_selected"] == out["n_above"] == int((out["dS"] > cfg.delta).sum())


def test_reset_writes_quasiequilibrium():
    """With beta = 0 the LBGK branch leaves f unchanged, so the output is the
    free flight of f with the selected sites replaced by f*."""
    cfg = oracle.make_cfg(Q=9, nx=9, ny=7, nu=INF, delta=1e-5, k=4)
    f = _near_eq_state(cfg, 8, amp=0.03)
    out = oracle.step(cfg, f)
    assert out["n_selected"] == 4
    post = f.copy()
    vx, vy, _ = oracle.velocities(9)
    for s in out["sel"]:
        y, x = divmod(int(s), cfg.nx)
        M = oracle.moments(9, f[:, y, x])
        post[:, y, x] = oracle.qe_poly(9, M[0], M[1] / M[0], M[2] / M[0])
    for i in range(9):
        assert np.array_equal(out["f"][i], np.roll(np.roll(post[i], vy[i], 0), vx[i], 1))


def test_uniform_free_stream_is_steady_in_channel():
    """Inlet equilibrium (west), zero-gradient (east), free-slip (south, north)."""
    for qe in (oracle.QE_POLY, oracle.QE_ENTROPIC_MM):
        cfg = oracle.make_cfg(Q=9, qe=qe, nx=12, ny=7, nu=1e-3,
                              bc=(W.INLET_EQ, W.ZEROGRAD, W.FREESLIP, W.FREESLIP),
                              inlet_rho=1.0, inlet_u=(0.05, 0.0))
        u = np.zeros((2, 7, 12))
        u[0] = 0.05
        f0 = oracle.init(cfg, np.ones((7, 12)), u)
        f = oracle.run(cfg, f0, 5)
        assert np.abs(f - f0).max() < 1e-15


def test_closed_box_conserves_mass():
    """Free-slip walls and a bounce-back square conserve mass exactly."""
    cfg = oracle.make_cfg(Q=9, nx=14, ny=10, nu=1e-2, delta=1e-4, k=3,
                          bc=(W.PERIODIC, W.PERIODIC, W.FREESLIP, W.FREESLIP), solid=(5, 3, 3, 4))
    f = _near_eq_state(cfg, 9)
    f[:, 3:7, 5:8] = 0.0
    m0 = f.sum()
    px0 = np.tensordot(oracle.velocities(9)[0], f, 1).sum()
    for _ in range(10):
        f = oracle.step(cfg, f)["f"]
    assert abs(f.sum() - m0) < 1e-12 * m0
    cfg2 = oracle.make_cfg(Q=9, nx=14, ny=10, nu=1e-2,
                           bc=(W.PERIODIC, W.PERIODIC, W.FREESLIP, W.FREESLIP))
    g = _near_eq_state(cfg2, 10)
    px0 = np.tensordot(oracle.velocities(9)[0], g, 1).sum()
    for _ in range(10):
        g = oracle.step(cfg2, g)["f"]
    # free-slip walls also conserve the wall-parallel momentum
    assert abs(np.tensordot(oracle.velocities(9)[0], g, 1).sum() - px0) < 1e-12


def test_inlet_and_bounce_back_values():
    cfg = oracle.make_cfg(Q=9, nx=10, ny=6, nu=INF,
                          bc=(W.INLET_EQ, W.ZEROGRAD, W.FREESLIP, W.FREESLIP),
                          inlet_rho=1.1, inlet_u=(0.05, 0.01), solid=(5, 2, 2, 2))
    f = _near_eq_state(cfg, 11)
    g = oracle.step(cfg, f)["f"]
    feq = oracle.qe_poly(9, 1.1, 0.05, 0.01)
    for i in (1, 5, 8):  # E, NE, SE enter through the west face (corners included)
        assert np.all(g[i, :, 0] == feq[i])
    # bounce-back: west of the solid, the W population is the E one returned
    assert g[3, 2, 4] == f[1, 2, 4]
    # free-slip at the top: S(x, top) = N(x, top)
    assert g[4, 5, 3] == f[2, 5, 3]


def _total_variation(rho, lo, hi):
    return float(np.abs(np.diff(rho[lo:hi])).sum())


def test_shock_tube_ehrenfest_subdues_oscillations():
    """Sec. 4.1: at nu = 1e-9 plain LBGK oscillates behind the shock; with
    Ehrenfests' steps at a few sites the oscillation is reduced."""
    base, rho, u = W.shock_tube()
    res = {}
    for name, k in (("lbgk", 0), ("es", 4)):
        cfg = oracle.cfg_from_dict(dict(base, k=k))
        f = oracle.init(cfg, rho, u[:1])
        n_sel = 0
        for _ in range(400):
            out = oracle.step(cfg, f)
            f = out["f"]
            n_sel += out["n_selected"]
        res[name] = (f.sum(0)[0], n_sel)
    tv_l = _total_variation(res["lbgk"][0], 250, 700)
    tv_e = _total_variation(res["es"][0], 250, 700)
    assert res["es"][1] > 0
    assert tv_e < tv_l


@pytest.mark.parametrize("qe", [oracle.QE_POLY, oracle.QE_ENTROPIC_M])
def test_step_at_sites_equals_whole_step(qe):
    """The per-site evaluation used on large lattices reproduces the whole
    step (same selection) at every site, boundaries and solid included."""
    cfg = oracle.make_cfg(Q=9, qe=qe, nx=23, ny=11, nu=1e-3, delta=1e-5, k=6,
                          bc=(W.INLET_EQ, W.ZEROGRAD, W.FREESLIP, W.FREESLIP),
                          inlet_rho=1.0, inlet_u=(0.05, 0.0), solid=(8, 4, 3, 3))
    f = _near_eq_state(cfg, 14, amp=0.02)
    f[:, 4:7, 8:11] = 0.0
    out = oracle.step(cfg, f)
    sites = np.arange(cfg.nx * cfg.ny)
    g = oracle.step_sites(cfg, f, sites, out["sel"])
    assert np.array_equal(g.T.reshape(out["f"].shape), out["f"])
    ds = oracle.site_dS(cfg, f, sites[:40])
    assert np.array_equal(ds, out["dS"].reshape(-1)[:40])


def test_elbm_step_conserves_entropy_at_beta_one():
    """ELBM with beta = 1 (nu = 0) replaces every f by its entropic
    involution, which keeps the entropy (Sec. 3.2); free flight keeps it too,
    so the total perfect entropy is unchanged, while LBGK changes it."""
    for Q, ny in ((3, 1), (9, 7)):
        cfg_e = oracle.make_cfg(Q=Q, qe=oracle.QE_ENTROPIC_MM, nx=15, ny=ny, nu=0.0,
                                collision=oracle.COLL_ELBM)
        cfg_l = oracle.make_cfg(Q=Q, qe=oracle.QE_ENTROPIC_MM, nx=15, ny=ny, nu=0.0)
        f = _near_eq_state(cfg_e, 15, amp=0.05)
        _, _, w = oracle.velocities(Q)
        S = lambda h: -np.sum(h * np.log(h / w[:, None, None]))
        se = S(oracle.step(cfg_e, f)["f"])
        sl = S(oracle.step(cfg_l, f)["f"])
        assert abs(se - S(f)) < 1e-12 * abs(S(f))
        assert abs(sl - S(f)) > 1e3 * abs(se - S(f))


def test_elbm_reduces_to_lbgk_near_equilibrium():
    cfg_e = oracle.make_cfg(Q=9, qe=oracle.QE_ENTROPIC_MM, nx=9, ny=5, nu=1e-3, collision=oracle.COLL_ELBM)
    cfg_l = oracle.make_cfg(Q=9, qe=oracle.QE_ENTROPIC_MM, nx=9, ny=5, nu=1e-3)
    for amp in (1e-2, 1e-3, 1e-4):
        f = _near_eq_state(cfg_e, 16, amp=amp)
        d = np.abs(oracle.step(cfg_e, f)["f"] - oracle.step(cfg_l, f)["f"]).max()
        assert d < 2 * amp * amp


def _np_step_outlet(cfg, f, Q):
    """The outlet channel step written independently with numpy: LBGK
    collision with the (separately pinned) polynomial quasiequilibrium,
    free flight by numpy.roll (periodic in y), then the inlet rule at x = 0
    and the outlet rule of Sec. 4.2 at x = nx - 1: the inward populations
    are the quasiequilibrium at the density and velocity of the new state of
    the penultimate column."""
    vx, vy, _ = oracle.velocities(Q)
    beta = 1.0 / (1.0 + 6.0 * cfg.nu)
    ny, nx = f.shape[1:]
    rho = f.sum(0)
    j1 = np.tensordot(vx, f, 1)
    j2 = np.tensordot(vy, f, 1)
    fs = np.zeros_like(f)
    for y in range(ny):
        for x in range(nx):
            fs[:, y, x] = oracle.qe_poly(Q, rho[y, x], j1[y, x] / rho[y, x], j2[y, x] / rho[y, x])
    post = f + 2.0 * beta * (fs - f)
    g = np.stack([np.roll(np.roll(post[i], vy[i], 0), vx[i], 1) for i in range(Q)])
    fin = oracle.qe_poly(Q, cfg.inlet_rho, cfg.inlet_u1, cfg.inlet_u2)
    for i in range(Q):
        if vx[i] > 0:
            g[i, :, 0] = fin[i]
    pen = g[:, :, nx - 2]
    for y in range(ny):
        r = pen[:, y].sum()
        fo = oracle.qe_poly(Q, r, np.dot(vx, pen[:, y]) / r, np.dot(vy, pen[:, y]) / r)
        for i in range(Q):
            if vx[i] < 0:
                g[i, y, nx - 1] = fo[i]
    return g


@pytest.mark.parametrize("Q", [3, 9])
def test_outlet_rule_matches_numpy_definition(Q):
    ny = 1 if Q == 3 else 5
    cfg = oracle.make_cfg(Q=Q, nx=9, ny=ny, nu=2e-3, bc=(W.INLET_EQ, W.OUTLET_EQ, W.PERIODIC, W.PERIODIC),
                          inlet_rho=1.05, inlet_u=(0.04, 0.0))
    r = np.random.default_rng(40 + Q)
    rho = 1 + 0.1 * r.uniform(-1, 1, (ny, 9))
    u = 0.08 * r.uniform(-1, 1, (2, ny, 9))
    f = oracle.init(cfg, rho, u[:1] if Q == 3 else u)
    f *= 1 + 0.03 * r.uniform(-1, 1, f.shape)
    got = oracle.step(cfg, f)["f"]
    want = _np_step_outlet(cfg, f, Q)
    assert np.abs(got - want).max() <= 1e-15 * np.abs(want).max()
    # the rule reads the new state of column nx - 2, not the old one
    vx = oracle.velocities(Q)[0]
    i = int(np.where(vx < 0)[0][0])
    old = f[:, 0, 7]
    stale = oracle.qe_poly(Q, old.sum(), np.dot(vx, old) / old.sum(), 0.0 if Q == 3 else
                           np.dot(oracle.velocities(Q)[1], old) / old.sum())[i]
    assert abs(got[i, 0, 8] - stale) > 1e-6
    # the other reading (OUTLET_EQ_PREV): the same step, except that every
    # inward population of the outlet column is the quasiequilibrium of the
    # old state of column nx - 2, whose density and velocity are typed here
    # from the moments of that state
    cp = oracle.make_cfg(Q=Q, nx=9, ny=ny, nu=2e-3, bc=(W.INLET_EQ, oracle.BC_OUTLET_EQ_PREV, W.PERIODIC, W.PERIODIC),
                         inlet_rho=1.05, inlet_u=(0.04, 0.0))
    gp = oracle.step(cp, f)["f"]
    vy = oracle.velocities(Q)[1]
    for yy in range(ny):
        old = f[:, yy, 7]
        r0 = old.sum()
        fe = oracle.qe_poly(Q, r0, np.dot(vx, old) / r0, 0.0 if Q == 3 else np.dot(vy, old) / r0)
        for q in np.where(vx < 0)[0]:
            assert abs(gp[q, yy, 8] - fe[q]) <= 1e-15 * r0
    inward = np.zeros(gp.shape, bool)
    inward[vx < 0, :, 8] = True
    assert np.array_equal(gp[~inward], got[~inward])


def test_outlet_corner_and_free_slip():
    """Corners: the x rule first (all three inward populations at the outlet
    corner come from the penultimate column's quasiequilibrium); a uniform
    free stream is steady with the outlet rule (poly and entropic QE)."""
    cfg = oracle.make_cfg(Q=9, nx=10, ny=6, nu=1e-3, bc=(W.INLET_EQ, W.OUTLET_EQ, W.FREESLIP, W.FREESLIP),
                          inlet_rho=1.0, inlet_u=(0.05, 0.0))
    f = _near_eq_state(cfg, 41, amp=0.02)
    g = oracle.step(cfg, f)["f"]
    for y in (0, 5):
        pen = g[:, y, 8]
        fo = oracle.qe_poly(9, pen.sum(), np.dot(oracle.velocities(9)[0], pen) / pen.sum(),
                            np.dot(oracle.velocities(9)[1], pen) / pen.sum())
        for i in (3, 6, 7):  # W, NW, SW enter through the east face
            assert abs(g[i, y, 9] - fo[i]) <= 1e-15
    for qe in (oracle.QE_POLY, oracle.QE_ENTROPIC_MM):
        c2 = oracle.make_cfg(Q=9, qe=qe, nx=12, ny=7, nu=1e-3,
                             bc=(W.INLET_EQ, W.OUTLET_EQ, W.FREESLIP, W.FREESLIP),
                             inlet_rho=1.0, inlet_u=(0.05, 0.0))
        u = np.zeros((2, 7, 12))
        u[0] = 0.05
        f0 = oracle.init(c2, np.ones((7, 12)), u)
        assert np.abs(oracle.run(c2, f0, 5) - f0).max() < 1e-15


def test_outlet_in_per_site_step():
    """The per-site step (used at full size) applies the outlet rule too."""
    d, rho, u, _ = W.cylinder_paper(1000.0, L=4, outlet=W.OUTLET_EQ)
    cfg = oracle.cfg_from_dict(dict(d, delta=1e-6))
    f = oracle.init(cfg, rho, u)
    r = np.random.default_rng(42)
    f *= 1 + 0.02 * r.uniform(-1, 1, f.shape)
    x0, y0, w, h = d["solid"]
    f[:, y0:y0 + h, x0:x0 + w] = 0.0
    out = oracle.step(cfg, f)
    assert out["n_selected"] == d["k"]
    nx, ny = d["nx"], d["ny"]
    sites = np.concatenate([np.arange(ny) * nx + nx - 1, np.arange(ny) * nx + nx - 2, np.arange(0, nx * ny, 17)])
    g = oracle.step_sites(cfg, f, sites, out["sel"])
    assert np.array_equal(g, out["f"].reshape(9, -1)[:, sites].T)


def test_conservation_sums_pins():
    """or_sums: a uniform state gives N_fluid x its moments (closed form);
    solid sites are left out; free flight on a periodic lattice (a
    permutation) leaves the sums unchanged; a step's reported input sums are
    the sums of its input; the mass and momentum of a periodic step with
    Ehrenfests' steps are conserved to round-off (Sec. 3.1, Sec. 3.2)."""
    rho, u1, u2 = 1.25, 0.0625, -0.03125
    cfg = oracle.make_cfg(Q=9, nx=12, ny=5, nu=1e-3, solid=(3, 1, 2, 2))
    fs = oracle.qe_poly(9, rho, u1, u2)
    f = np.repeat(fs[:, None], 60, axis=1).reshape(9, 5, 12).copy()
    f[:, 1:3, 3:5] = 7.0                   # solid sites hold anything: not counted
    s = oracle.sums(cfg, f)
    nfl = 60 - 4
    # polynomial QE (cited D2Q9 form): 2E = rho (2/3 + |u|^2)
    want = [nfl * rho, nfl * rho * u1, nfl * rho * u2, nfl * rho * (2.0 / 3.0 + u1 * u1 + u2 * u2)]
    assert np.allclose(s, want, rtol=1e-14, atol=1e-14)
    # D1Q3: no y momentum
    c3 = oracle.make_cfg(Q=3, nx=7, ny=1)
    f3 = np.repeat(oracle.qe_poly(3, 0.5, 0.1)[:, None], 7, axis=1).reshape(3, 1, 7)
    assert np.allclose(oracle.sums(c3, f3), [3.5, 0.35, 0.0, 7 * 0.5 * (1.0 / 3.0 + 0.01)], rtol=1e-14)
    # free flight is a permutation of each plane
    cp = oracle.make_cfg(Q=9, nx=13, ny=7, nu=INF)
    g = _near_eq_state(cp, 21)
    h = oracle.step(cp, g)["f"]
    assert np.allclose(oracle.sums(cp, h), oracle.sums(cp, g), rtol=1e-15, atol=1e-15)
    # the step's input sums, and conservation with resets
    cq = oracle.make_cfg(Q=9, nx=11, ny=6, nu=1e-3, delta=1e-4, k=5)
    g = _near_eq_state(cq, 22)
    o = oracle.step(cq, g)
    assert np.allclose(o["sums"], oracle.sums(cq, g), rtol=1e-14, atol=1e-14)
    assert o["n_selected"] > 0
    a, b = oracle.sums(cq, g), oracle.sums(cq, o["f"])
    assert np.abs(a[:3] - b[:3]).max() < 1e-13 * a[0]
