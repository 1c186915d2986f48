"""Non-finite halt: the first time step that meets non-finite populations
stops every later step kernel, so the last finite state is kept; the
library then reports LBM_E_NONFINITE and hands back that state and its step
number (the plain LBGK divergence that Sec. 4.2 reports for the unregularised
scheme is the case this serves).  Nothing faults: the values overflow in
ordinary FP32 arithmetic."""
import math

import numpy as np
import pytest

import workloads as W
from _gpu_common import lattice, say, torch_gpu

pytestmark = pytest.mark.gpu


def _unstable(nx=64, ny=32, u0=0.5):
    """Plain LBGK at nu = 0 (beta = 1) with a fast uniform stream: linearly
    unstable, it overflows FP32 within about a hundred steps."""
    n = nx * ny
    rho = np.ones((ny, nx))
    u = np.zeros((2, ny, nx))
    u[0] = u0 + 1e-3 * W.noise(41, 1, n).reshape(ny, nx)
    u[1] = 0.02 * np.sin(2 * math.pi * np.arange(nx) / nx)[None, :]
    d = dict(Q=9, qe=W.QE_POLY, nx=nx, ny=ny, nu=0.0, delta=math.inf, k=0, bc=(W.PERIODIC,) * 4)
    return d, rho, u


def test_halt_keeps_last_finite_state():
    torch = torch_gpu()
    import paper_0705_4371_amd.lbm as lbm
    d, rho, u = _unstable()
    say("case halt: unstable LBGK 64x32 fp32")
    a = lattice(d, 0, rho, u)
    a.step(300)                  # graph replays and direct launches
    st, _, _ = a.stats()
    say("  halted", st.nonfinite, "last finite step", st.step)
    assert st.nonfinite == 1 and 10 < st.step < 299
    fa = a.get_populations()
    assert bool(torch.isfinite(fa).all())
    with pytest.raises(lbm.LbmError) as e:
        a.step(1)
    assert e.value.code == lbm.LBM_E_NONFINITE
    # the kept state is the state after exactly st.step steps
    b = lattice(d, 0, rho, u)
    b.step(st.step)
    sb, _, _ = b.stats()
    assert sb.nonfinite == 0 and sb.step == st.step
    assert torch.equal(b.get_populations(), fa)
    # one more step is the one that fails, at the same step number
    b.step(1)
    sb, _, _ = b.stats()
    assert sb.nonfinite == 1 and sb.step == st.step
    assert torch.equal(b.get_populations(), fa)
    # new populations clear the halt
    a.set_populations(fa)
    a.step(1)
    sa, _, _ = a.stats()
    assert sa.nonfinite == 1 and sa.step == 0   # the same failing step, from the canonical layout
    assert torch.equal(a.get_populations(), fa)
    a.close()
    b.close()


def test_halt_reported_by_step_without_stats():
    torch = torch_gpu()
    import paper_0705_4371_amd.lbm as lbm
    d, rho, u = _unstable()
    say("case halt: lbm_step reports it")
    a = lattice(d, 0, rho, u)
    a.step(300)
    torch.cuda.synchronize()     # the host copy of the halt word has landed
    with pytest.raises(lbm.LbmError) as e:
        a.step(1)
    assert e.value.code == lbm.LBM_E_NONFINITE
    st, _, _ = a.stats()
    assert st.nonfinite == 1
    a.close()


def test_halt_on_first_step_from_canonical_state():
    """A density that overflows FP32 at one site: the very first step (which
    reads the canonical layout) halts; the state set is kept bit for bit."""
    torch = torch_gpu()
    d, rho, u = W.shear_layer(nx=64, ny=16, k=4, delta=1e-4, width=5.0)
    say("case halt: first step, rho overflow")
    lat = lattice(d, 0, rho, u)
    f = lat.get_populations()
    f[1:5, 7, 9] = 1.0e38        # finite populations whose sum is not
    lat.set_populations(f)
    lat.step(5)
    st, _, _ = lat.stats()
    assert st.nonfinite == 1 and st.step == 0
    assert torch.equal(lat.get_populations(), f)
    lat.close()


def test_halt_in_fstarM_step():
    """The same halt through the f*_M time step (solve, fallback and
    collision in k_fstep): a site whose populations are about to overflow."""
    torch = torch_gpu()
    import paper_0705_4371_amd.lbm as lbm
    nx, ny = 64, 16
    d, rho, u = W.shear_layer(nx=nx, ny=ny, k=4, delta=1e-4, width=5.0)
    d = dict(d, qe=W.QE_ENTROPIC_M)
    e0 = W.iso_energy(u[0], u[1])
    say("case halt: f*_M step")
    lat = lattice(d, 0, rho, u, twoE0=e0)
    lat.step(3)
    f = lat.get_populations()
    f[1:5, 3, 20] = 1.0e38
    lat.set_populations(f)
    lat.step(40)
    st, _, _ = lat.stats()
    assert st.nonfinite == 1 and st.step == 0
    assert torch.equal(lat.get_populations(), f)
    with pytest.raises(lbm.LbmError):
        lat.step(1)
    lat.close()
