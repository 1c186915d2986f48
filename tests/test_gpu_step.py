"""GPU parity of the Ehrenfests'-regularised step (through the C-ABI) with
the CPU oracle, teacher-forced: each GPU step starts from the GPU state, and
the oracle takes one step from exactly those populations.

Bars: FP64 populations within 1e-12 of the oracle relative to max |f|,
FP32 within 1e-5; FP64 Delta S of every candidate within 1e-12 relative to
max(Delta S, delta); candidate and selected sets identical except at sites
whose Delta S lies within 1e-12 of delta or of the k-th value.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from _gpu_common import compare_step, lattice, perturb, say, torch_gpu

pytestmark = pytest.mark.gpu

FP32, FP64 = 0, 1
TOL = {FP32: 1e-5, FP64: 1e-12}


def _run(d, rho, u, prec, seed, amp, nsteps=3, label=""):
    torch = torch_gpu()
    say("case", label, d["Q"], d["nx"], d["ny"], "prec", prec, "k", d.get("k"), "delta", d.get("delta"))
    lat = lattice(d, prec, rho, u)
    f0 = lat.get_populations().double().cpu().numpy()
    f0 = perturb(f0, seed, amp, d.get("solid"))
    lat.set_populations(torch.from_numpy(f0))
    f = lat.get_populations().double().cpu().numpy()   # rounded to the context precision
    out = []
    for s in range(nsteps):
        g, o, st = compare_step(lat, d, f, TOL[prec], label="%s step %d" % (label, s))
        out.append((g, o, st))
        f = g
    lat.close()
    return out


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_shock_tube_teacher_forced(prec):
    d, rho, u = W.shock_tube()
    _run(d, rho, u[:1], prec, 1, 0.05, nsteps=4, label="shock")


def test_shock_tube_400_steps_fp64():
    """The full shock-tube run, every step teacher-forced."""
    torch = torch_gpu()
    d, rho, u = W.shock_tube()
    say("case shock 400")
    lat = lattice(d, FP64, rho, u[:1])
    f = lat.get_populations().double().cpu().numpy()
    n_sel = 0
    for s in range(400):
        g, o, st = compare_step(lat, d, f, 1e-12, label="shock400 step %d" % s)
        n_sel += st.n_selected
        f = g
    assert n_sel > 0
    lat.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
@pytest.mark.parametrize("k", [0, 5, 40, 100000])
def test_periodic_shear_small(prec, k):
    d, rho, u = W.shear_layer(nx=300, ny=70, k=k, delta=1e-4, width=20.0)
    _run(d, rho, u, prec, 2, 0.02, label="shear k=%d" % k)


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_cylinder_channel_small(prec):
    d, rho, u = W.cylinder(nx=530, ny=48, side=10, centre=(120, 24), re=200.0, delta=1e-5, k=30)
    _run(d, rho, u, prec, 3, 0.02, label="cylinder")


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_entropic_mm_qe(prec):
    d, rho, u = W.shear_layer(nx=260, ny=33, k=12, delta=1e-5, width=10.0)
    d = dict(d, qe=W.QE_ENTROPIC_MM)
    _run(d, rho, u, prec, 4, 0.03, label="entropic-mm")


def test_ties_and_forced_radix_path():
    """Many identical sites (exact Delta S ties) and n_above >> k."""
    torch = torch_gpu()
    d, rho, u = W.shear_layer(nx=200, ny=40, k=37, delta=1e-6, width=5.0)
    lat = lattice(d, FP64, rho, u)
    f = perturb(lat.get_populations().double().cpu().numpy(), 5, 0.01)
    # columns of identical sites: rows 3..30 of column 17 copy site (17, 2)
    f[:, 3:31, 17] = f[:, 2:3, 17]
    f[:, 3:31, 150] = f[:, 2:3, 17]
    lat.set_populations(torch.from_numpy(f))
    g, o, st = compare_step(lat, d, f, 1e-12, label="ties")
    assert o["n_above"] > 5 * d["k"]
    lat.close()


def test_delta_zero_all_sites_candidates():
    d, rho, u = W.shear_layer(nx=130, ny=20, k=64, delta=0.0, width=5.0)
    out = _run(d, rho, u, FP64, 6, 0.01, nsteps=2, label="delta0")
    assert out[0][2].n_above_delta == 130 * 20


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_delta_s_series_orders_mixed_in_a_wavefront(prec):
    """The FP64 Delta S of a population is its short series (|s| <= 1/16), its
    long series (|s| <= 1/4) or the logarithm, and a wavefront evaluates one
    series for all its lanes only when every lane allows it.  Perturbation
    amplitudes cycling through 0.02, 0.3 and 0.9 along x put lanes that need
    each form into every wavefront (64 consecutive sites); with delta = 0
    every site is a candidate and its Delta S is held to the oracle's."""
    torch = torch_gpu()
    d, rho, u = W.shear_layer(nx=192, ny=8, k=64, delta=0.0, width=5.0)
    say("case mixed series orders prec", prec)
    lat = lattice(d, prec, rho, u)
    f0 = lat.get_populations().double().cpu().numpy()
    r = np.random.default_rng(17)
    amp = np.array([0.02, 0.3, 0.9])[np.arange(d["nx"]) % 3]
    f0 = f0 * (1 + amp[None, None, :] * r.uniform(-1, 1, f0.shape))
    lat.set_populations(torch.from_numpy(f0))
    f = lat.get_populations().double().cpu().numpy()
    g, o, st = compare_step(lat, d, f, TOL[prec], label="mixed series orders")
    assert st.n_above_delta == d["nx"] * d["ny"]
    lat.close()


def test_invalid_sites_rank_first():
    torch = torch_gpu()
    d, rho, u = W.shear_layer(nx=128, ny=16, k=6, delta=1e-5, width=5.0)
    lat = lattice(d, FP64, rho, u)
    f = perturb(lat.get_populations().double().cpu().numpy(), 7, 0.01)
    f[3, 5, 40] = -1e-3      # negative population
    f[1, 9, 100] = -2e-3
    lat.set_populations(torch.from_numpy(f))
    g, o, st = compare_step(lat, d, f, 1e-12, label="invalid")
    assert st.n_invalid == 2
    _, sel, ds = lat.stats(sel_cap=6)
    assert math.isinf(ds[0]) and math.isinf(ds[1]) and sel[0] < sel[1]
    lat.close()


def test_graph_replay_matches_direct_launches():
    """64 steps through the captured graphs equal 64 directly launched steps
    bit for bit, and the last step still matches the oracle."""
    torch = torch_gpu()
    d, rho, u = W.cylinder(nx=300, ny=60, side=12, centre=(80, 30), re=300.0, delta=1e-4, k=16)
    a = lattice(d, FP32, rho, u)
    b = lattice(d, FP32, rho, u)
    f0 = perturb(a.get_populations().double().cpu().numpy(), 8, 0.02, d["solid"])
    a.set_populations(torch.from_numpy(f0))
    b.set_populations(torch.from_numpy(f0))
    b.set_timing(True)           # timing mode launches kernels directly
    a.step(65)
    b.step(65)
    ga = a.get_populations().cpu().numpy()
    gb = b.get_populations().cpu().numpy()
    assert np.array_equal(ga, gb)
    sa, _, _ = a.stats()
    sb, _, _ = b.stats()
    assert sa.total_selected == sb.total_selected and sa.step == sb.step == 65
    ms, n = b.kernel_time()
    assert n == 65 and ms > 0
    f = a.get_populations().double().cpu().numpy()
    compare_step(a, d, f, 1e-5, label="after graphs")
    a.close()
    b.close()


def test_deterministic_repeat():
    torch = torch_gpu()
    d, rho, u = W.shear_layer(nx=256, ny=64, k=50, delta=1e-5, width=20.0)
    res = []
    for _ in range(2):
        lat = lattice(d, FP32, rho, u)
        f0 = perturb(lat.get_populations().double().cpu().numpy(), 9, 0.02)
        lat.set_populations(torch.from_numpy(f0))
        lat.step(5)
        res.append((lat.get_populations().cpu().numpy(), lat.stats(sel_cap=50)))
        lat.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1][1], res[1][1][1])


def test_moments_and_init():
    torch = torch_gpu()
    d, rho, u = W.cylinder(nx=140, ny=30, side=6, centre=(40, 15), re=100.0)
    for prec in (FP64, FP32):
        lat = lattice(d, prec, rho, u)
        g = lat.get_populations().double().cpu().numpy()
        want = oracle.init(oracle.cfg_from_dict(d), rho, u)
        tol = 1e-15 if prec == FP64 else 1e-7
        assert np.abs(g - want).max() <= tol * np.abs(want).max()
        r, ru, e2 = (t.cpu().numpy() for t in lat.moments())
        vx, vy, _ = oracle.velocities(9)
        assert np.abs(r - g.sum(0)).max() < 1e-13
        assert np.abs(ru[0] - np.tensordot(vx, g, 1)).max() < 1e-13
        assert np.abs(ru[1] - np.tensordot(vy, g, 1)).max() < 1e-13
        assert np.abs(e2 - np.tensordot(vx * vx + vy * vy, g, 1)).max() < 1e-13
        lat.close()


def test_nonfinite_rejected():
    torch = torch_gpu()
    import paper_0705_4371_amd.lbm as lbm
    d, rho, u = W.shear_layer(nx=64, ny=8, k=2, delta=1e-4, width=5.0)
    lat = lattice(d, FP32, rho, u)
    f = lat.get_populations()
    f[2, 3, 4] = float("nan")
    with pytest.raises(lbm.LbmError) as e:
        lat.set_populations(f)
    assert e.value.code == lbm.LBM_E_NONFINITE
    with pytest.raises(lbm.LbmError):
        lat.step(1)
    lat.close()


def _fstarM_case(nx=240, ny=44):
    d, rho, u = W.cylinder(nx=nx, ny=ny, side=8, centre=(60, ny // 2), re=300.0, delta=1e-5, k=16,
                           qe=W.QE_ENTROPIC_M)
    n = nx * ny
    e0 = W.iso_energy(u[0], u[1]) * (1.0 + 0.02 * W.noise(31, 0, n).reshape(ny, nx))
    return d, rho, u, e0


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_entropic_fstarM_in_step(prec):
    """The f*_M quasiequilibrium inside the step (moments -> per-site Newton ->
    collide / rank / reset), teacher-forced against the oracle's FP64 solve."""
    torch = torch_gpu()
    d, rho, u, e0 = _fstarM_case()
    say("case fstarM step prec", prec)
    lat = lattice(d, prec, rho, u, twoE0=e0)
    g0 = lat.get_populations().double().cpu().numpy()
    want = oracle.init(oracle.cfg_from_dict(d), rho, u, e0)
    assert np.abs(g0 - want).max() <= (1e-12 if prec == FP64 else 2e-7) * np.abs(want).max()
    f = perturb(g0, 12, 0.02, d["solid"])
    lat.set_populations(torch.from_numpy(f))
    f = lat.get_populations().double().cpu().numpy()
    tol = 1e-12 if prec == FP64 else 1e-5
    for s in range(3):
        g, o, st = compare_step(lat, d, f, tol, label="fstarM step %d" % s)
        assert st.newton_updates > 0 and st.n_fallback == o["n_fallback"] == 0
        assert st.n_failed == 0 and st.max_resid <= (1e-13 if prec == FP64 else 1e-10)
        f = g
    lat.close()


@pytest.mark.parametrize("start,prec", [("closed", FP32), ("prev", FP64), ("prev", FP32)])
def test_entropic_fstarM_step_starts(start, prec):
    """The closed-form and previous-step starts of the f*_M solve inside the
    step give the oracle's step (the start changes the iterations only)."""
    torch = torch_gpu()
    import paper_0705_4371_amd.lbm as lbm
    d, rho, u, e0 = _fstarM_case()
    st0 = lbm.LBM_START_CLOSED_FORM if start == "closed" else lbm.LBM_START_PREV
    say("case fstarM step start", start, "prec", prec)
    lat = lattice(d, prec, rho, u, twoE0=e0, fstar_start=st0)
    f = perturb(lat.get_populations().double().cpu().numpy(), 14, 0.02, d["solid"])
    lat.set_populations(torch.from_numpy(f))
    f = lat.get_populations().double().cpu().numpy()
    tol = 1e-12 if prec == FP64 else 1e-5
    for s in range(3):
        g, o, st = compare_step(lat, d, f, tol, label="fstarM %s step %d" % (start, s))
        assert st.newton_updates > 0 and st.n_fallback == 0
        assert st.n_failed == 0 and st.max_resid <= (1e-13 if prec == FP64 else 1e-10)
        f = g
    lat.close()


@pytest.mark.parametrize("budget,target", [((0, 1), 1e-13), ((2, 1), 1e-10)])
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_entropic_fstarM_step_fallback(prec, budget, target):
    """First-pass budgets too small for the residual target: the sites that
    miss it (all of them with (0, 1)) are solved by the damped fallback and
    collided there; the step still matches the oracle.  In FP64 contexts
    every converged solve, the fallback's included, takes one more Newton
    update (to round-off), so even a 1e-10 target meets the 1e-12 bound."""
    torch = torch_gpu()
    d, rho, u, e0 = _fstarM_case(nx=200, ny=36)
    say("case fstarM fallback budget", budget, "target", target, "prec", prec)
    lat = lattice(d, prec, rho, u, twoE0=e0)
    lat.set_fstar_tolerance(tol=target, max32=budget[0], max64=budget[1])
    f = perturb(lat.get_populations().double().cpu().numpy(), 15, 0.02, d["solid"])
    lat.set_populations(torch.from_numpy(f))
    f = lat.get_populations().double().cpu().numpy()
    tol = 1e-12 if prec == FP64 else 1e-5
    n_fluid = d["nx"] * d["ny"] - int(np.prod(d["solid"][2:]))
    for s in range(2):
        g, o, st = compare_step(lat, d, f, tol, label="fstarM fallback %s step %d" % (budget, s))
        say("  fallbacks", st.n_fallback, "of", n_fluid, "max residual", st.max_resid)
        assert st.n_fallback > 0 and st.n_failed == 0
        assert st.max_resid <= (1e-13 if prec == FP64 else target)
        if budget == (0, 1):
            assert st.n_fallback >= 0.99 * n_fluid
        f = g
    lat.close()


@pytest.mark.parametrize("start", ["rest", "prev"])
def test_fstarM_graph_replay_matches_direct_launches(start):
    """The fused f*_M step (solve, collision, fallback and the statistics
    clear inside the captured graphs): three rounds of 32 graph-replayed
    steps, each checked bit for bit against as many directly launched steps
    after the host has read the state back, then one step against the
    oracle."""
    torch = torch_gpu()
    import paper_0705_4371_amd.lbm as lbm
    d, rho, u, e0 = _fstarM_case(nx=200, ny=36)
    st0 = lbm.LBM_START_DEFAULT if start == "rest" else lbm.LBM_START_PREV
    say("case fstarM graph replay start", start)
    a = lattice(d, FP32, rho, u, twoE0=e0, fstar_start=st0)
    b = lattice(d, FP32, rho, u, twoE0=e0, fstar_start=st0)
    f0 = perturb(a.get_populations().double().cpu().numpy(), 18, 0.02, d["solid"])
    a.set_populations(torch.from_numpy(f0))
    b.set_populations(torch.from_numpy(f0))
    a.step(1)                    # the first step after set_populations is direct in both
    b.step(1)
    b.set_timing(True)           # timing mode launches kernels directly
    for r in range(3):
        a.step(32)
        b.step(32)
        ga = a.get_populations().cpu().numpy()
        gb = b.get_populations().cpu().numpy()
        assert np.array_equal(ga, gb), "replay round %d" % r
        sa, _, _ = a.stats()
        sb, _, _ = b.stats()
        assert (sa.total_selected, sa.newton_updates, sa.n_fallback) == \
            (sb.total_selected, sb.newton_updates, sb.n_fallback), "replay round %d" % r
        say("  round", r, "selected", sa.total_selected, "updates", sa.newton_updates)
    f = a.get_populations().double().cpu().numpy()
    compare_step(a, d, f, 1e-5, label="fstarM after graphs")
    a.close()
    b.close()


def test_elbm_fstarM_fallback_fp64():
    """ELBM with the f*_M quasiequilibrium and every site forced through the
    damped fallback, whose collision then takes the ELBM alpha."""
    torch = torch_gpu()
    d, rho, u, e0 = _fstarM_case(nx=200, ny=36)
    d = dict(d, collision=1)
    say("case elbm fstarM fallback")
    lat = lattice(d, FP64, rho, u, twoE0=e0)
    lat.set_fstar_tolerance(tol=1e-13, max32=0, max64=1)
    f = perturb(lat.get_populations().double().cpu().numpy(), 19, 0.02, d["solid"])
    lat.set_populations(torch.from_numpy(f))
    f = lat.get_populations().double().cpu().numpy()
    n_fluid = d["nx"] * d["ny"] - int(np.prod(d["solid"][2:]))
    for s in range(2):
        g, o, st = compare_step(lat, d, f, 1e-12, label="elbm fstarM fallback step %d" % s)
        assert st.n_fallback >= 0.99 * n_fluid and st.n_failed == 0
        f = g
    lat.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_elbm_with_fstarM(prec):
    """ELBM (eq. elbmLB) with the f*_M quasiequilibrium and Ehrenfests' steps
    on the small cylinder channel."""
    torch = torch_gpu()
    d, rho, u, e0 = _fstarM_case()
    d = dict(d, collision=1)
    say("case elbm fstarM prec", prec)
    lat = lattice(d, prec, rho, u, twoE0=e0)
    f = perturb(lat.get_populations().double().cpu().numpy(), 16, 0.02, d["solid"])
    lat.set_populations(torch.from_numpy(f))
    f = lat.get_populations().double().cpu().numpy()
    tol = 1e-12 if prec == FP64 else 1e-5
    for s in range(2):
        g, o, st = compare_step(lat, d, f, tol, label="elbm fstarM step %d" % s)
        assert st.n_failed == 0
        f = g
    lat.close()


def test_entropic_fstarM_network_start_with_fallback():
    """An untrained network start: the warm-started Newton pass misses the
    tolerance at many sites, the plain-Newton fallback re-solves them, and the
    step still matches the oracle."""
    torch = torch_gpu()
    import paper_0705_4371_amd.lbm as lbm
    d, rho, u, e0 = _fstarM_case(nx=200, ny=36)
    net = lbm.Mlp(3)
    ish, isc, osh, _ = W.mlp_norm()
    net.set_norm(ish, isc, osh, [0.05] * 4)   # a deliberately poor start: O(10) multiplier errors
    lat = lattice(d, FP64, rho, u, twoE0=e0, fstar_start=lbm.LBM_START_MLP, net=net)
    f = perturb(lat.get_populations().double().cpu().numpy(), 13, 0.02, d["solid"])
    lat.set_populations(torch.from_numpy(f))
    f = lat.get_populations().double().cpu().numpy()
    g, o, st = compare_step(lat, d, f, 1e-12, label="fstarM net start")
    say("  fallbacks", st.n_fallback)
    assert st.n_fallback > 0 and st.n_failed == 0
    lat.close()
    net.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_elbm_shock_tube(prec):
    """ELBM (eq. elbmLB) with Ehrenfests' steps on the shock tube (the
    configuration of Fig. 1 (i): entropic QE, nu = 1e-9, (k, delta) = (4, 1e-4))."""
    d, rho, u = W.shock_tube(delta=1e-4)
    d = dict(d, qe=W.QE_ENTROPIC_MM, collision=1)
    _run(d, rho, u[:1], prec, 17, 0.05, nsteps=4, label="elbm shock")


def test_elbm_shock_tube_400_steps_fp64():
    torch = torch_gpu()
    d, rho, u = W.shock_tube(delta=1e-4)
    d = dict(d, qe=W.QE_ENTROPIC_MM, collision=1)
    lat = lattice(d, FP64, rho, u[:1])
    f = lat.get_populations().double().cpu().numpy()
    for s in range(400):
        g, o, st = compare_step(lat, d, f, 1e-12, label="elbm400 step %d" % s)
        f = g
    lat.close()


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_elbm_d2q9(prec):
    d, rho, u = W.shear_layer(nx=140, ny=30, k=9, delta=1e-5, width=8.0)
    d = dict(d, qe=W.QE_ENTROPIC_MM, collision=1)
    _run(d, rho, u, prec, 18, 0.03, label="elbm d2q9")


SELECT_CASES = {
    "ties, n >> k": lambda: W.shear_layer(nx=200, ny=40, k=37, delta=1e-6, width=5.0),
    "delta 0": lambda: W.shear_layer(nx=130, ny=20, k=64, delta=0.0, width=5.0),
    "n < k": lambda: W.shear_layer(nx=96, ny=16, k=5000, delta=1e-5, width=5.0),
    "k 0": lambda: W.shear_layer(nx=96, ny=16, k=0, delta=1e-5, width=5.0),
    "cylinder": lambda: W.cylinder(nx=240, ny=80, side=16, centre=(60, 40), re=5000.0, k=9, delta=1e-5),
}


@pytest.mark.parametrize("name", list(SELECT_CASES))
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_select_paths_agree(name, prec):
    """The one-workgroup and the multi-workgroup ranking and selection give
    bit-identical populations, selected sets and statistics (and both match
    the oracle)."""
    torch = torch_gpu()
    d, rho, u = SELECT_CASES[name]()
    say("case select paths", name, "prec", prec)
    runs = []
    for mode in (1, 2):
        lat = lattice(d, prec, rho, u, select_mode=mode)
        f = perturb(lat.get_populations().double().cpu().numpy(), 71, 0.01, d.get("solid"))
        if name == "ties, n >> k":
            f[:, 3:31, 17] = f[:, 2:3, 17]
        lat.set_populations(torch.from_numpy(f))
        f = lat.get_populations().double().cpu().numpy()
        res = []
        for s in range(2):
            g, o, st = compare_step(lat, d, f, TOL[prec], label="%s mode %d step %d" % (name, mode, s))
            _, sel, sel_ds = lat.stats(sel_cap=max(d["k"], 1))
            res.append((g, sel, sel_ds, st.n_above_delta, st.n_selected, st.n_invalid, st.kth_dS, st.max_dS))
            f = g
        runs.append(res)
        lat.close()
    for (a, b) in zip(runs[0], runs[1]):
        assert np.array_equal(a[0], b[0])
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        assert a[3:] == b[3:]
