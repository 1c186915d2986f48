"""FP64 conservation sums (mass and momentum, Sec. 3.1; a reset to f* keeps
the moments, Sec. 3.2; 2E) of free-running GPU trajectories against the FP64
oracle's own trajectory from the same initial state, and their drift.  The
figures are printed for the design notes."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from _gpu_common import lattice, say, torch_gpu

pytestmark = pytest.mark.gpu


def _trajectory(d, rho, u, prec, nsteps, every, e0=None):
    torch = torch_gpu()
    lat = lattice(d, prec, rho, u, twoE0=e0)
    f0 = lat.get_populations().double().cpu().numpy()
    gpu = []
    for t in range(0, nsteps + 1, every):
        if t:
            lat.step(every)
        st, _, _ = lat.stats()
        assert st.nonfinite == 0 and st.step == t
        gpu.append([st.mass, st.mom[0], st.mom[1], st.energy])
    lat.close()
    oc = oracle.cfg_from_dict(d)
    f = f0
    orc = [oracle.sums(oc, f)]
    for t in range(1, nsteps + 1):
        f = oracle.step(oc, f)["f"]
        if t % every == 0:
            orc.append(oracle.sums(oc, f))
    return np.array(gpu), np.array(orc)


def _report(label, g, o):
    m0 = o[0, 0]
    dev = np.abs(g - o).max(axis=0) / m0
    drift_g = np.abs(g - g[0]).max(axis=0) / m0
    drift_o = np.abs(o - o[0]).max(axis=0) / m0
    say("  %s: GPU vs oracle (mass, mom1, mom2, 2E) / mass: %s" % (label, " ".join("%.2e" % v for v in dev)))
    say("  %s: drift GPU %s | oracle %s" % (label, " ".join("%.2e" % v for v in drift_g),
                                           " ".join("%.2e" % v for v in drift_o)))
    return dev, drift_g, drift_o


def test_shock_tube_400_steps_sums():
    d, rho, u = W.shock_tube()
    say("case conservation: shock tube 800, 400 steps, fp64")
    g, o = _trajectory(d, rho, u[:1], 1, 400, 50)
    dev, dg, do = _report("shock fp64", g, o)
    assert dev.max() <= 1e-12
    # mass is conserved to round-off on both sides (the waves have not reached
    # the zero-gradient ends); momentum is not: the two ends hold different
    # pressures, (rho_L - rho_R) c_s^2 = 1/6 per step, 400/6 after 400 steps
    assert dg[0] <= 1e-13 and do[0] <= 1e-13
    assert abs(o[-1, 1] / o[0, 0] - (400.0 / 6.0) / 600.0) < 1e-3


@pytest.mark.parametrize("prec", [1, 0])
def test_periodic_shear_sums(prec):
    d, rho, u = W.shear_layer(nx=128, ny=64, width=80.0 * 64 / 4096 * 8, k=16, delta=1e-6)
    say("case conservation: shear 128x64, 300 steps, prec", prec)
    g, o = _trajectory(d, rho, u, prec, 300, 50)
    dev, dg, do = _report("shear %s" % ("fp64" if prec else "fp32"), g, o)
    if prec == 1:
        assert dev.max() <= 1e-12
        assert dg[:3].max() <= 1e-13
    else:
        # FP32 storage: each stored population is rounded to 2^-24 of itself,
        # so a step moves the mass by at most 2^-24 of it (the same bound for
        # the momentum and 2E sums relative to the mass); the drift is below
        # steps x 2^-24
        bound = 300 * 2.0 ** -24
        assert dev.max() <= bound and dg[:3].max() <= bound
    assert do[:3].max() <= 1e-13


def test_fstarM_sums_conserve_energy():
    """With f*_M the collision also conserves 2E (the energy row is one of
    the constraints of Sec. 2's argmax)."""
    nx, ny = 96, 48
    d, rho, u = W.shear_layer(nx=nx, ny=ny, width=10.0, k=8, delta=1e-6)
    d = dict(d, qe=W.QE_ENTROPIC_M)
    e0 = W.iso_energy(u[0], u[1]) * (1.0 + 0.02 * W.noise(43, 0, nx * ny).reshape(ny, nx))
    say("case conservation: f*_M shear 96x48, 100 steps, fp64")
    g, o = _trajectory(d, rho, u, 1, 100, 25, e0=e0)
    dev, dg, do = _report("fstarM fp64", g, o)
    assert dev.max() <= 1e-12
    assert dg.max() <= 1e-12 and do.max() <= 1e-12
