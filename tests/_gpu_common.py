"""Shared helpers of the GPU parity tests: build the GPU context from a
workload dict, run teacher-forced steps, and compare with the oracle."""
import math
import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stderr.flush()


def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def lattice(d, precision, rho, u, stream=None, twoE0=None, fstar_start=0, net=None, select_mode=0):
    import paper_0705_4371_amd.lbm as lbm
    cfg = lbm.config_from_workload(d, precision, stream=stream, fstar_start=fstar_start, net=net,
                                   select_mode=select_mode)
    return lbm.Lattice(cfg, rho, u, twoE0)


def perturb(f, seed, amp, solid=None):
    r = np.random.default_rng(seed)
    g = f * (1 + amp * r.uniform(-1, 1, f.shape))
    if solid is not None and solid[2] > 0:
        x0, y0, w, h = solid
        g[:, y0:y0 + h, x0:x0 + w] = 0.0
    return g


def exempt_sites(o_dS, delta, kth, rel=1e-12):
    """Sites whose FP64 Delta S lies within rel of delta or of the k-th value."""
    d = o_dS.reshape(-1)
    ex = np.zeros(d.size, bool)
    for ref in (delta, kth):
        if ref is None or not math.isfinite(ref) or ref <= 0:
            continue
        ex |= np.abs(d - ref) <= rel * np.maximum(np.abs(d), ref)
    return ex


def compare_step(lat, d, f_in, tol, label=""):
    """One GPU step from the current GPU state (whose canonical populations
    are f_in, float64 numpy) against one oracle step from f_in."""
    oc = oracle.cfg_from_dict(d)
    o = oracle.step(oc, f_in)
    lat.step(1)
    g = lat.get_populations().double().cpu().numpy()
    st, sel, sel_ds = lat.stats(sel_cap=max(d.get("k", 0), 1))
    k = d.get("k", 0)
    delta = d.get("delta", math.inf)
    # candidate set and Delta S
    sites, ds = lat.candidates()
    o_dS = o["dS"].reshape(-1)
    o_cand = np.flatnonzero(o_dS > delta)
    ex = exempt_sites(o_dS, delta, float(o_dS[o["sel"][-1]]) if len(o["sel"]) else None)
    gset, oset = set(sites.tolist()), set(o_cand.tolist())
    diff = np.array(sorted(gset ^ oset), dtype=np.int64)
    assert ex[diff].all() if diff.size else True, "%s candidate sets differ at %s" % (label, diff[:10])
    if sites.size:
        ref = o_dS[sites]
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(ds), fin), label
        scale = np.maximum(ref[fin], delta if math.isfinite(delta) else 0.0)
        err = np.abs(ds[fin] - ref[fin]) / np.maximum(scale, 1e-300)
        assert err.max(initial=0.0) <= 1e-12, "%s Delta S rel err %g" % (label, err.max())
    # selected set
    sdiff = np.array(sorted(set(sel.tolist()) ^ set(o["sel"].tolist())), dtype=np.int64)
    assert st.n_selected == min(k, o["n_above"]) == o["n_selected"], (label, st.n_selected, o["n_selected"])
    assert st.n_above_delta == o["n_above"] or ex[diff].all(), label
    if sdiff.size:
        assert ex[sdiff].all(), "%s selected sets differ at %s" % (label, sdiff[:10])
    # rank order of the report: Delta S descending, ties by site
    if sel.size > 1:
        keys = list(zip((-sel_ds).tolist(), sel.tolist()))
        assert keys == sorted(keys), label
    # populations: mask destinations of exempt disagreements
    mask = np.ones(g.shape, bool)
    if sdiff.size:
        vx, vy, _ = oracle.velocities(d["Q"])
        for s in sdiff:
            y, x = divmod(int(s), d["nx"])
            for i in range(d["Q"]):
                mask[i, (y + vy[i]) % d["ny"], (x + vx[i]) % d["nx"]] = False
    scale = np.abs(o["f"]).max()
    err = np.abs(g - o["f"])[mask].max() / scale
    assert err <= tol, "%s population rel err %g > %g" % (label, err, tol)
    # FP64 conservation sums of f(t+1) computed on the GPU (Sec. 3.1: the
    # collision conserves mass and momentum; Sec. 3.2: a reset keeps the
    # moments) against the FP64 oracle's sums of its own f(t+1): 1e-12 of
    # the mass in FP64 contexts, 1e-6 in FP32 (the FP32 step's rounding of
    # the populations; the summation itself is FP64 on both sides)
    fp64 = lat.cfg.precision == 1
    sums = np.array([st.mass, st.mom[0], st.mom[1], st.energy])
    want = oracle.sums(oc, o["f"])
    own = oracle.sums(oc, g)
    err = np.abs(sums - want) / want[0]
    SUMS_ERR.append((label, "fp64" if fp64 else "fp32", err.max()))
    assert err.max() <= (1e-12 if fp64 else 1e-6), (label, sums, want, err)
    # the GPU's summation order against the oracle's on the same populations
    assert np.abs(sums - own).max() <= 1e-13 * own[0], (label, sums, own)
    return g, o, st


# (label, precision, max relative error of the four conservation sums
# against the oracle) of every compare_step of the session
SUMS_ERR = []
