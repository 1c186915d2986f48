"""Edge cases of the step on the GPU against the oracle (teacher-forced,
bars as in test_gpu_step.py): degenerate lattices (2 x 2, 3 x 1, a single
row), k larger than the lattice, every site a candidate, a lattice of one
64-site tile, widths that leave ragged tiles; and, at the full 8192 x 4096
size, an outbreak with every site above delta (33.5 million candidates, so
that every ranking workgroup flushes its LDS histogram several times), whose
selection is checked against a sort of the GPU's own candidate keys and
whose Delta S and populations are checked against the oracle at sampled
sites."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from _gpu_common import compare_step, lattice, perturb, say, torch_gpu

pytestmark = pytest.mark.gpu
FP32, FP64 = 0, 1
TOL = {FP32: 1e-5, FP64: 1e-12}


def _uniform(nx, ny, seed, Q=9, umax=0.05):
    r = np.random.default_rng(seed)
    rho = 1 + 0.05 * r.uniform(-1, 1, (ny, nx))
    u = umax * r.uniform(-1, 1, (2, ny, nx))
    return rho, (u[:1] if Q == 3 else u)


CASES = {
    "2x2 periodic, delta 0, k 1": (dict(Q=9, nx=2, ny=2, nu=1e-3, delta=0.0, k=1), 0.02),
    "2x2 periodic, k 100 > N": (dict(Q=9, nx=2, ny=2, nu=1e-3, delta=1e-7, k=100), 0.02),
    "3x1 D1Q3 inlet/outlet, k 5 > N": (dict(Q=3, nx=3, ny=1, nu=1e-3, delta=1e-7, k=5,
                                            bc=(W.INLET_EQ, W.OUTLET_EQ, W.PERIODIC, W.PERIODIC),
                                            inlet_rho=1.02, inlet_u=(0.03, 0.0)), 0.02),
    "3x2 free-slip, zero-gradient": (dict(Q=9, nx=3, ny=2, nu=1e-2, delta=1e-6, k=2,
                                          bc=(W.ZEROGRAD, W.ZEROGRAD, W.FREESLIP, W.FREESLIP)), 0.03),
    "one row 300x1 D2Q9": (dict(Q=9, nx=300, ny=1, nu=1e-4, delta=1e-6, k=7), 0.02),
    "one tile 64x1 D1Q3 entropic": (dict(Q=3, qe=W.QE_ENTROPIC_MM, nx=64, ny=1, nu=1e-5, delta=1e-6, k=3), 0.02),
    "ragged 65x3, k = N": (dict(Q=9, nx=65, ny=3, nu=1e-3, delta=1e-6, k=195), 0.02),
    "ragged 257x5 channel, outlet": (dict(Q=9, qe=W.QE_ENTROPIC_MM, nx=257, ny=5, nu=1e-4, delta=1e-6, k=9,
                                          bc=(W.INLET_EQ, W.OUTLET_EQ, W.FREESLIP, W.FREESLIP),
                                          inlet_rho=1.0, inlet_u=(0.05, 0.0)), 0.02),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", [FP64, FP32])
def test_degenerate_lattices(name, prec):
    torch = torch_gpu()
    d, amp = CASES[name]
    say("case", name, "prec", prec)
    rho, u = _uniform(d["nx"], d["ny"], 50 + len(name), Q=d["Q"])
    lat = lattice(d, prec, rho, u)
    f = perturb(lat.get_populations().double().cpu().numpy(), 60 + len(name), amp)
    lat.set_populations(torch.from_numpy(f))
    f = lat.get_populations().double().cpu().numpy()
    for s in range(3):
        g, o, st = compare_step(lat, d, f, TOL[prec], label="%s step %d" % (name, s))
        assert st.n_selected == min(d["k"], o["n_above"])
        f = g
    lat.close()


def test_outbreak_every_site_full_size():
    torch = torch_gpu()
    say("case outbreak 8192 x 4096 FP32, every site perturbed")
    d, rho, u = W.shear_layer()
    lat = lattice(d, FP32, rho, u)
    del rho, u
    f = lat.get_populations()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(12)
    f *= 1 + 0.05 * (2 * torch.rand(f.shape, generator=gen, device="cuda", dtype=torch.float32) - 1)
    lat.set_populations(f)
    del f
    fh = lat.get_populations().double().cpu().numpy()
    oc = oracle.cfg_from_dict(d)
    lat.step(1)
    st, sel, sel_ds = lat.stats(sel_cap=d["k"])
    sites, ds = lat.candidates()
    N = d["nx"] * d["ny"]
    say("  candidates %d of %d, selected %d" % (sites.size, N, sel.size))
    # more than 512 workgroups x 256 x 128 screened sites: every ranking
    # workgroup flushes its LDS histogram at least once mid-run
    assert sites.size > 512 * 256 * 128 and st.n_selected == d["k"] == sel.size
    assert np.unique(sites).size == sites.size
    # the selection is the top k of the candidates' keys (Delta S desc, site asc)
    order = np.lexsort((sites, -ds))[:d["k"]]
    assert set(sites[order].tolist()) == set(sel.tolist())
    assert st.kth_dS == ds[order[-1]] and st.max_dS == ds.max()
    # candidate Delta S against the oracle at sampled candidates, including the selected
    r = np.random.default_rng(13)
    probe = np.concatenate([r.integers(0, sites.size, 1500), order[:100]])
    ods = oracle.site_dS(oc, fh, sites[probe])
    fin = np.isfinite(ods)
    assert np.array_equal(np.isfinite(ds[probe]), fin)
    err = np.abs(ds[probe][fin] - ods[fin]) / np.maximum(ods[fin], d["delta"])
    assert err.max() <= 1e-12, err.max()
    # no false negatives among sampled non-candidates
    cand = np.zeros(N, bool)
    cand[sites] = True
    others = np.flatnonzero(~cand)
    if others.size:
        pick = others[r.integers(0, others.size, min(2000, others.size))]
        assert (oracle.site_dS(oc, fh, pick) <= d["delta"] * (1 + 1e-12)).all()
    # populations at sampled output sites, with the GPU's selected set
    g = lat.get_populations()
    out_sites = np.unique(np.concatenate([r.integers(0, N, 1500), sel[:200]]))
    want = oracle.step_sites(oc, fh, out_sites, sel)
    got = g.reshape(9, -1)[:, torch.from_numpy(out_sites).cuda()].double().cpu().numpy().T
    e = np.abs(got - want).max() / np.abs(want).max()
    say("  sampled population rel err %.3g" % e)
    assert e <= 1e-5
    lat.close()
