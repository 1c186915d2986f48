#!/usr/bin/env python3
"""Throughput of the Ehrenfests'-regularised LBGK time step on one MI355X.

Workload (default): the doubly periodic D2Q9 double shear layer,
8192 x 4096 sites, FP32 populations, polynomial quasiequilibrium,
nu = 1e-6, delta = 1e-4, k = 4096 -- the HBM-bound configuration whose
throughput is reported in MLUPS and against the HBM roofline.  A "step" is
one full time step: fused stream/collide with Delta S screening, FP64
ranking of the screened sites, top-k selection and the Ehrenfests' reset.

Prints one JSON line:
  value      MLUPS (fluid sites x steps / s) over the timed steps
  roofline   the fused step kernel (k_step): algorithmic bytes per launch
             (72 B per site in FP32, 144 B in FP64: every population read
             once and written once) / its mean launch duration, measured
             with HIP events on the context's stream around the step kernel
             of every timed step
  cpu_baseline  the CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def traffic_from_profile(workload: str, prec: str, n_sites: int):
    """HBM bytes per k_step launch from the committed rocprofv3 PMC summary,
    or None if the summary is missing or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "k_step_%s_%s_pmc.json" % (workload, prec))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    from paper_0705_4371_amd.profiling import kernel_source_hash
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def host_cpu():
    """CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "cores_available": cores, "nproc": os.cpu_count()}


def _oracle_rate(oracle, cfg, f, steps, omp):
    t0 = time.perf_counter()
    for _ in range(steps):
        f = oracle.step(cfg, f, omp=omp)["f"]
    return time.perf_counter() - t0


def cpu_baseline(args, net_params=None):
    """The oracle (FP64 C) timed on this host: the plain single-threaded
    build (the parity reference) and the same source built with OpenMP over its
    site loops, on bounded samples of the workloads (see `sample`)."""
    import numpy as np
    import oracle
    import workloads as W
    host = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", host["cores_available"]))
    oracle.build(force=False, omp=True)
    out = {"unit": "MLUPS", "kind": "oracle", "host": host}
    # the headline workload: row bands of the shear layer (same nu, delta, k)
    d, rho, u = W.shear_layer(nx=args.cpu_nx, ny=args.cpu_rows, width=80.0 * args.cpu_rows / 4096)
    cfg = oracle.cfg_from_dict(d)
    f = oracle.init(cfg, rho, u)
    n = args.cpu_nx * args.cpu_rows
    dt_omp = _oracle_rate(oracle, cfg, f, args.cpu_steps, True)
    d1, rho1, u1 = W.shear_layer(nx=args.cpu_nx, ny=args.cpu_rows // 2, width=80.0 * (args.cpu_rows // 2) / 4096)
    cfg1 = oracle.cfg_from_dict(d1)
    f1 = oracle.init(cfg1, rho1, u1)
    dt1 = _oracle_rate(oracle, cfg1, f1, 2, False)
    out["value"] = n * args.cpu_steps / dt_omp / 1e6
    out["cores"] = threads
    out["sample"] = ("%d x %d band of the 8192 x 4096 shear layer, %d steps, FP64, OpenMP build on %d threads, "
                     "%.1f s" % (args.cpu_nx, args.cpu_rows, args.cpu_steps, threads, dt_omp))
    out["single_thread"] = {"value": args.cpu_nx * (args.cpu_rows // 2) * 2 / dt1 / 1e6, "unit": "MLUPS",
                            "cores": 1, "sample": "%d x %d band, 2 steps, plain build, %.1f s"
                                                  % (args.cpu_nx, args.cpu_rows // 2, dt1)}
    # the 1-D shock tube in full (800 sites, 400 steps, FP64)
    d, rho, u = W.shock_tube()
    cfg = oracle.cfg_from_dict(d)
    f = oracle.init(cfg, rho, u[:1])
    dts = _oracle_rate(oracle, cfg, f, 400, False)
    out["shock_tube_800"] = {"steps": 400, "seconds": round(dts, 3), "MLUPS": round(800 * 400 / dts / 1e6, 3),
                             "cores": 1}
    # the 1200 x 400 square-cylinder channel (Re 1000): a few steps
    d, rho, u = W.CONFIGS["cylinder_1200x400_re1000"]()
    cfg = oracle.cfg_from_dict(d)
    f = oracle.init(cfg, rho, u)
    dtc = _oracle_rate(oracle, cfg, f, args.cpu_channel_steps, True)
    mc = 480000 * args.cpu_channel_steps / dtc / 1e6
    out["channel_1200x400"] = {"steps": args.cpu_channel_steps, "seconds": round(dtc, 3), "MLUPS": round(mc, 3),
                               "cores": threads, "extrapolated_50k_steps_s": round(50000 * 480000 / (mc * 1e6), 1)}
    # f*_M of the 4096 x 2048 moment field to residual 1e-10 (the whole
    # field from the rest and closed-form starts; the network start, whose
    # forward pass the oracle runs on one thread, on an evenly spaced sample)
    Mf = W.moment_field()
    M = Mf[:, ::max(1, Mf.shape[1] // args.cpu_fstar_sites)][:, :args.cpu_fstar_sites].copy()
    ns = M.shape[1]
    fst = {"sites": ns, "cores": threads, "residual": 1e-10}
    for name, start in (("rest", 0), ("closed_form", 1)):
        t0 = time.perf_counter()
        _, it, bad = oracle.fstar_field(M, 1e-10, start, omp=True)
        dtf = time.perf_counter() - t0
        fst[name] = {"Msites_per_s": round(ns / dtf / 1e6, 3), "mean_newton_updates": round(float(it.mean()), 3),
                     "unconverged": bad, "seconds": round(dtf, 2)}
    del Mf
    if net_params is not None:
        # the network start in FP64 (forward pass on the oracle), then Newton
        M = M[:, ::max(1, ns // args.cpu_mlp_sites)][:, :args.cpu_mlp_sites].copy()
        ns = M.shape[1]
        fst["mlp_sites"] = ns
        nm = np.concatenate(W.mlp_norm()).astype(np.float32)
        t0 = time.perf_counter()
        y = oracle.mlp_forward(net_params.astype(np.float64), oracle.mlp_features(M, nm))
        mu = oracle.mlp_unnormalise(y, nm)
        mu[0] += np.log(M[0])
        _, it, bad = oracle.fstar_field(M, 1e-10, 2, mu=mu, omp=True)
        dtf = time.perf_counter() - t0
        fst["mlp"] = {"Msites_per_s": round(ns / dtf / 1e6, 3), "mean_newton_updates": round(float(it.mean()), 3),
                      "unconverged": bad, "note": "FP64 forward pass of the trained network on one thread"}
    out["fstar_4096x2048"] = fst
    return out


def settle(lat, torch, seconds):
    """Untimed steps for `seconds` (the GPU clocks settle before timing)."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        lat.step(64)
        torch.cuda.synchronize()


def timed_steps(lat, torch, nsteps):
    """`nsteps` directly launched steps with HIP events around every step
    kernel.  Returns (wall seconds, summed kernel ms, timed launches)."""
    lat.set_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.step(nsteps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    ms, n = lat.kernel_time()
    lat.set_timing(False)
    return wall, ms, n


def fp64_leg(args, torch, lbm, W):
    """The same shear layer with FP64 populations (144 B per site and step):
    whole-step rate and the step kernel's HBM roofline from the same timed
    steps (HIP events around every step kernel)."""
    d, rho, u = W.shear_layer(nx=args.nx, ny=args.ny)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        lat = lbm.Lattice(lbm.config_from_workload(d, lbm.LBM_FP64, stream=stream.cuda_stream), rho, u)
    del rho, u
    n_sites = args.nx * args.ny
    lat.step(args.warmup)
    torch.cuda.synchronize()
    settle(lat, torch, args.settle_s)
    dt, k_ms, k_n = timed_steps(lat, torch, args.fp64_steps)
    ms_step = dt * 1e3 / args.fp64_steps
    k_avg_ms = k_ms / max(k_n, 1)
    assert k_n == args.fp64_steps and k_ms <= dt * 1e3, ("inconsistent timing", k_ms, dt * 1e3)
    st, _, _ = lat.stats()
    lat.close()
    ach = 144 * n_sites / (k_avg_ms / 1e3) / 1e9
    return {"steps": args.fp64_steps, "MLUPS": round(n_sites * args.fp64_steps / dt / 1e6, 1),
            "ms_per_step": round(ms_step, 4),
            "roofline": {"bound": "hbm", "kernel": "k_step", "kernel_ms": round(k_avg_ms, 4),
                         "kernel_launches": k_n, "bytes_per_site": 144, "achieved": round(ach, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4)},
            "nonfinite": st.nonfinite}


def cylinder_leg(args, torch, lbm, W, net, solver=None):
    """Flow past the square cylinder on 2400 x 800 at Re = 20000 with the
    entropic f*_M quasiequilibrium in every step (per-site Newton, plain-Newton
    fallback) and Ehrenfests' steps (delta = 1e-3, k = 256), from the rest
    start and from the trained network start.  With a solver, the solve of
    the moments of every fluid site after the rest-start run's last step is
    timed from each start as on the moment field (the network start's gain
    on the cylinder's own distribution)."""
    d, rho, u = W.CONFIGS["cylinder_2400x800_re20000_fstarM"]()
    e0 = W.iso_energy(u[0], u[1])
    out = {"lattice": "%dx%d" % (d["nx"], d["ny"]), "steps": max(1, args.cyl_steps // 1000) * min(1000, max(1, args.cyl_steps)),
           "sampling": "the statistics of every 1000th step"}
    for name, start in (("rest", lbm.LBM_START_DEFAULT), ("mlp", lbm.LBM_START_MLP),
                        ("previous_step", lbm.LBM_START_PREV)):
        cfg = lbm.config_from_workload(d, lbm.LBM_FP32, fstar_start=start,
                                       net=net if start == lbm.LBM_START_MLP else None)
        lat = lbm.Lattice(cfg, rho, u, e0)
        lat.step(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fb = 0
        upd = 0
        above = 0
        failed = 0
        maxres = 0.0
        chunk = min(1000, max(1, args.cyl_steps))
        nch = max(1, args.cyl_steps // chunk)
        done, nonfinite = 0, 0
        for _ in range(nch):
            lat.step(chunk)
            st, _, _ = lat.stats()
            if st.nonfinite:
                nonfinite = 1
                break
            done += 1
            fb += st.n_fallback
            upd += st.newton_updates
            above += st.n_above_delta
            failed += st.n_failed
            maxres = max(maxres, st.max_resid)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nch = max(done, 1)
        st, _, ds = lat.stats(sel_cap=256)
        fluid = d["nx"] * d["ny"] - d["solid"][2] * d["solid"][3]
        out[name] = {"steps_run": int(st.step), "nonfinite": nonfinite,
                     "MLUPS": round(fluid * nch * chunk / dt / 1e6, 1),
                     "ms_per_step": round(dt * 1e3 / (nch * chunk), 4),
                     "fallback_sites_sampled_steps": int(fb),
                     "fallback_rate": fb / (fluid * nch),
                     "newton_updates_per_site": upd / (fluid * nch),
                     "failed_sites_sampled_steps": int(failed), "max_residual_sampled_steps": maxres,
                     "mean_n_above_delta_sampled": round(above / nch, 2),
                     "last_step": {"n_above_delta": st.n_above_delta, "n_selected": st.n_selected,
                                   "max_dS": st.max_dS, "kth_dS": st.kth_dS, "nonfinite": st.nonfinite},
                     "selected_total": st.total_selected, "mass": st.mass, "energy": st.energy}
        if name == "rest" and solver is not None and not nonfinite:
            import numpy as np
            rho_t, ru_t, e2_t = lat.moments()
            x0, y0, w, h = d["solid"]
            solid = np.zeros((d["ny"], d["nx"]), bool)
            solid[y0:y0 + h, x0:x0 + w] = True
            fl = torch.from_numpy(np.flatnonzero(~solid.reshape(-1))).cuda()
            Mc = torch.stack([rho_t.reshape(-1), ru_t[0].reshape(-1), ru_t[1].reshape(-1),
                              e2_t.reshape(-1)]).index_select(1, fl).contiguous()
            del rho_t, ru_t, e2_t, fl
            out["field_solve"] = {"field": "moments of the %d fluid sites after step %d of the rest-start run"
                                           % (Mc.shape[1], int(st.step)),
                                  "solve": _solve_starts(torch, lbm, solver, Mc, net)}
            del Mc
        lat.close()
        # every sampled step reached the residual target at every site
        assert failed == 0 and maxres <= 1e-10, (name, failed, maxres)
    return out


def channel_leg(args, torch, lbm, W):
    """Flow past the square cylinder on 1200 x 400 (side 40 centred at
    (300, 200), inlet u = (0.05, 0), zero-gradient outlet, free-slip walls,
    polynomial QE, FP32, delta = 1e-3, k = 64) at Re = 1000, 5000 and 20000,
    each for the full run length, through the step graphs; the Ehrenfests'
    statistics (and the FP64 sums behind them) are read every `chunk` steps."""
    out = {"lattice": "1200x400", "steps": args.channel_steps, "precision": "fp32"}
    chunk = 1000
    for re in (1000, 5000, 20000):
        d, rho, u = W.CONFIGS["cylinder_1200x400_re%d" % re]()
        cfg = lbm.config_from_workload(d, lbm.LBM_FP32)
        lat = lbm.Lattice(cfg, rho, u)
        lat.step(20)
        torch.cuda.synchronize()
        print("# channel Re = %d: %d steps" % (re, args.channel_steps), file=sys.stderr, flush=True)
        above = 0
        samples = 0
        t0 = time.perf_counter()
        done = 0
        nonfinite_in = None
        last_finite = None
        while done < args.channel_steps:
            n = min(chunk, args.channel_steps - done)
            lat.step(n)
            done += n
            st, _, _ = lat.stats()
            if st.nonfinite:
                # the run diverged in this chunk; the library kept the state
                # of the last finite step, whose number stats report
                nonfinite_in = [done - n, done]
                last_finite = st.step
                break
            above += st.n_above_delta
            samples += 1
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sites = d["nx"] * d["ny"]
        r = {"steps_run": done, "MLUPS": round(sites * done / dt / 1e6, 1),
             "ms_per_step": round(dt * 1e3 / done, 5),
             "mean_n_above_delta_sampled": round(above / max(samples, 1), 2),
             "selected_total": st.total_selected, "nonfinite_in_steps": nonfinite_in,
             "last_finite_step": last_finite}
        if nonfinite_in is None:
            r["mass"] = st.mass
        out["re%d" % re] = r
        lat.close()
    return out


def active_leg(args, torch, lbm, lat, n_sites):
    """The same lattice with an outbreak of non-equilibrium: populations of a
    band of `rows` rows multiplied by 1 + 0.05 xi (xi uniform in [-1, 1),
    seeded), so that Delta S > delta at about 10^6 sites per step and the
    ranking, top-k selection (k = 4096 of n >> k) and reset run at full load.
    Timed over `steps` steps (whole step, wall clock)."""
    import numpy as np
    f = lat.get_populations()
    rows = args.active_rows
    y0 = (lat.cfg.ny - rows) // 2
    r = np.random.default_rng(11)
    band = torch.from_numpy(1 + 0.05 * r.uniform(-1, 1, (lat.Q, rows, lat.cfg.nx))).to(f.dtype).cuda()
    f[:, y0:y0 + rows, :] *= band
    lat.set_populations(f)
    del f, band
    lat.step(2)
    torch.cuda.synchronize()
    above = 0
    sel = 0
    chunk = 32  # one replay of the captured step graph per chunk
    dt = 0.0
    for _ in range(args.active_steps // chunk):
        t0 = time.perf_counter()
        lat.step(chunk)
        torch.cuda.synchronize()
        dt += time.perf_counter() - t0
        # the statistics (and the FP64 sums behind them) outside the timing
        st, _, _ = lat.stats()
        above += st.n_above_delta
        sel += st.n_selected
    nsamp = args.active_steps // chunk
    steps = nsamp * chunk
    return {"band_rows": rows, "steps": steps, "MLUPS": round(n_sites * steps / dt / 1e6, 1),
            "ms_per_step": round(dt * 1e3 / steps, 4),
            "mean_n_above_delta": round(above / nsamp, 1), "mean_n_selected": round(sel / nsamp, 1),
            "note": "wall clock of the steps, in chunks of %d; the statistics read after each chunk "
                    "is not timed" % chunk}


def _train_net(args, torch, lbm, W, solver, wide):
    """A warm-start network trained on 2^pairs_log2 (moments, multipliers)
    pairs of the study's distribution (wide: |u| <= 0.3, energy +-30%), the
    multipliers from the solver, the pairs built by the library."""
    npairs = 1 << args.pairs_log2
    kw = dict(umax=0.3, energy_band=0.3) if wide else {}
    Mtr = torch.from_numpy(W.random_moments(npairs, 5, **kw)).cuda()
    mu_tr, _, _, st = solver.solve(Mtr, start=lbm.LBM_START_DEFAULT)
    net = lbm.Mlp(5)
    net.set_norm(*W.mlp_norm(wide=wide))
    X, T = net.pairs(Mtr, mu_tr)
    del Mtr, mu_tr
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = net.train(X, T, epochs=args.epochs, batch=args.batch, lr=1e-3, seed=5)
    torch.cuda.synchronize()
    info = {"pairs": npairs, "epochs": args.epochs, "batch": args.batch,
            "adam_steps": args.epochs * (npairs // args.batch),
            "seconds": round(time.perf_counter() - t0, 3),
            "loss_first_epoch": float(losses[0]), "loss_last_epoch": float(losses[-1])}
    del X, T
    return net, info


def _time_gpu(torch, fn, reps=20):
    """Mean ms of fn() over reps back-to-back calls (HIP events on torch's
    current stream, which the library's default-stream calls share)."""
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4  # wave64 vector instructions per second (256 CUs x 4 SIMDs, 4 cycles each)


def _fstar_counts():
    """Vector instruction counts per 64 sites of the solver and network-start
    kernels on the 4096 x 2048 field, from the committed counter summary,
    while the hash of those kernels' sources recorded there still matches."""
    path = os.path.join(ROOT, "profiles", "fstar_kernels_4096x2048_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    from paper_0705_4371_amd.profiling import fstar_source_hash
    return d["kernels"] if d.get("fstar_source_hash") == fstar_source_hash() else None


def _update_hist(it, st):
    """Newton updates per site (the solver's histogram of the first pass) and
    the largest count of each wavefront (64 consecutive sites), which sets
    the wavefront's time, as {updates: number of sites / wavefronts}."""
    import numpy as np
    per_site = {str(j) if j < 15 else "15+": int(c) for j, c in enumerate(st.iter_hist) if c}
    u = it.cpu().numpy()
    nw = u.size // 64
    wmax = np.bincount(u[:nw * 64].reshape(nw, 64).max(axis=1))
    return {"updates_per_site_hist": per_site,
            "updates_per_wave_max_hist": {str(j): int(c) for j, c in enumerate(wmax) if c}}


def _solve_starts(torch, lbm, solver, M, net, counts=None):
    """Times the f*_M solve of the field M from the rest, closed-form and
    network starts, the network start's forward alone, and the solve from
    the exact multipliers (previous-state start at the converged solution:
    the fixed cost that no start removes)."""
    n = M.shape[1]
    mu = torch.empty_like(M)
    it = torch.empty(n, dtype=torch.uint8, device="cuda")
    stt = torch.empty(n, dtype=torch.uint8, device="cuda")
    res = {}
    # half a second of solves first, so that every start is timed at the
    # same (ramped) clocks
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.5:
        for _ in range(10):
            solver.solve(M, start=lbm.LBM_START_DEFAULT, stats=False, mu=mu, iters=it, status=stt)
        torch.cuda.synchronize()
    for name, start in (("plain_newton", lbm.LBM_START_PLAIN), ("rest", lbm.LBM_START_DEFAULT),
                        ("closed_form", lbm.LBM_START_CLOSED_FORM), ("mlp", lbm.LBM_START_MLP)):
        kw = dict(start=start, net=net if start == lbm.LBM_START_MLP else None, mu=mu, iters=it, status=stt)
        _, _, _, st = solver.solve(M, stats=True, **kw)          # statistics (synchronising)
        ms = _time_gpu(torch, lambda: solver.solve(M, stats=False, **kw))
        res[name] = {"ms": round(ms, 4), "Msites_per_s": round(n / ms / 1e3, 1),
                     "mean_newton_updates": round(st.mean_fp32_iters + st.mean_fp64_iters, 4),
                     "mean_fp32": round(st.mean_fp32_iters, 4), "mean_fp64": round(st.mean_fp64_iters, 4),
                     "fallback": int(st.n_fallback), "failed": int(st.n_failed),
                     "max_residual": st.max_resid}
    warm = torch.empty((4, n), dtype=torch.float32, device="cuda")
    res["mlp"]["forward_ms"] = round(_time_gpu(torch, lambda: net.warm_start(M, out=warm)), 4)
    # exact start: the converged multipliers as the previous-state start
    solver.solve(M, start=lbm.LBM_START_DEFAULT, stats=False, mu=mu, iters=it, status=stt)
    kw = dict(start=lbm.LBM_START_PREV, mu=mu, iters=it, status=stt)
    _, _, _, st = solver.solve(M, stats=True, **kw)
    ms = _time_gpu(torch, lambda: solver.solve(M, stats=False, **kw))
    res["exact_start"] = {"ms": round(ms, 4), "mean_fp32": round(st.mean_fp32_iters, 4),
                          "mean_fp64": round(st.mean_fp64_iters, 4), "failed": int(st.n_failed),
                          "max_residual": st.max_resid}
    # update histograms, after every timing (their host work would let the
    # clocks drop before the next timed solve)
    for name, start in (("plain_newton", lbm.LBM_START_PLAIN), ("rest", lbm.LBM_START_DEFAULT),
                        ("closed_form", lbm.LBM_START_CLOSED_FORM), ("mlp", lbm.LBM_START_MLP)):
        _, _, _, st = solver.solve(M, stats=True, start=start, net=net if start == lbm.LBM_START_MLP else None,
                                   mu=mu, iters=it, status=stt)
        res[name].update(_update_hist(it, st))
    # HBM floor of each solve: M read (32 B/site), mu written (32 B), the
    # update count and status bytes (2 B), and the network start read back
    # (16 B), or the previous multipliers (32 B) for the exact start; the
    # forward reads M and writes the start (48 B)
    for name, b in (("plain_newton", 66), ("rest", 66), ("closed_form", 66), ("mlp", 82), ("exact_start", 98)):
        res[name]["hbm_bytes_per_site"] = b
        res[name]["hbm_frac"] = round(b * n / (res[name]["ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
    res["mlp"]["forward_hbm_frac"] = round(48 * n / (res["mlp"]["forward_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
    # vector issue: counted instructions over the issue slots of the measured time
    if counts:
        for name, key, ms in (("plain_newton", "plain_newton", "ms"), ("rest", "rest", "ms"),
                              ("closed_form", "closed_form", "ms"),
                              ("exact_start", "exact_start", "ms"), ("mlp", "mlp_forward", "forward_ms")):
            if key in counts:
                c = counts[key]
                frac = c["valu"] * (n / 64.0) / (res[name][ms] * 1e-3) / VALU_ISSUE_PER_S
                res[name]["forward_issue_frac" if key == "mlp_forward" else "issue_frac"] = round(frac, 4)
        if "mlp" in counts:
            solve_ms = res["mlp"]["ms"] - res["mlp"]["forward_ms"]
            res["mlp"]["issue_frac"] = round(counts["mlp"]["valu"] * (n / 64.0) / (solve_ms * 1e-3)
                                             / VALU_ISSUE_PER_S, 4)
        res["issue_counts"] = "profiles/fstar_kernels_4096x2048_pmc.json (instructions per 64 sites)"
    # the method's own comparison: the network start against plain FP64
    # Newton from the default start (the fallback solve, run everywhere)
    for name in ("mlp", "rest", "closed_form", "exact_start"):
        res["speedup_%s_vs_plain_newton" % name] = round(res["plain_newton"]["ms"] / res[name]["ms"], 3)
    res["speedup_mlp_vs_rest"] = round(res["rest"]["ms"] / res["mlp"]["ms"], 3)
    res["speedup_closed_form_vs_rest"] = round(res["rest"]["ms"] / res["closed_form"]["ms"], 3)
    res["speedup_bound_any_start"] = round(res["rest"]["ms"] / res["exact_start"]["ms"], 3)
    return res


def fstar_leg(args, torch, lbm, W):
    """Entropic f*_M solve on the 4096 x 2048 moment field: the warm-start MLP
    is trained on 2^24 (moments, multipliers) pairs produced by the solver
    (batch 65536, 20 epochs, Adam 1e-3), then the solve is timed from the rest
    start, the closed-form start and the network start, each to a residual
    <= 1e-10 (plain Newton fallback enabled), beside plain FP64 Newton from
    the default start at every site (the reference the network start is
    measured against), the network forward alone and the exact start.  The same on a wide field (|u| <= 0.3, energy
    +-30%) with a network trained on that distribution."""
    out = {}
    solver = lbm.FstarSolver(max(1 << args.pairs_log2, args.fx * args.fy))
    net, out["training"] = _train_net(args, torch, lbm, W, solver, wide=False)
    M = torch.from_numpy(W.moment_field(nx=args.fx, ny=args.fy)).cuda()
    out["sites"] = M.shape[1]
    out["solve"] = _solve_starts(torch, lbm, solver, M, net, counts=_fstar_counts())
    del M
    if not args.no_cylinder:
        out["cylinder_fstarM"] = cylinder_leg(args, torch, lbm, W, net, solver)
    out["speedup_mlp_vs_plain_newton"] = out["solve"]["speedup_mlp_vs_plain_newton"]
    out["speedup_mlp_vs_rest"] = out["solve"]["speedup_mlp_vs_rest"]
    out["speedup_closed_form_vs_rest"] = out["solve"]["speedup_closed_form_vs_rest"]
    params = net.get_params()
    net.close()
    if not args.no_wide:
        wnet, winfo = _train_net(args, torch, lbm, W, solver, wide=True)
        Mw = torch.from_numpy(W.moment_field(nx=args.fx, ny=args.fy, umax=0.3, energy_band=0.3)).cuda()
        out["wide"] = {"field": "4096x2048 smooth, |u| <= 0.3, 2E/rho within 30% of isothermal",
                       "training": winfo, "solve": _solve_starts(torch, lbm, solver, Mw, wnet)}
        del Mw
        wnet.close()
    solver.close()
    return out, params


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--nx", type=int, default=8192)
    ap.add_argument("--ny", type=int, default=4096)
    ap.add_argument("--settle-s", type=float, default=1.0,
                    help="seconds of untimed steps after the warm-up steps (clock ramp)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 shear-layer leg")
    ap.add_argument("--fp64-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-nx", type=int, default=8192)
    ap.add_argument("--cpu-rows", type=int, default=512)
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--cpu-channel-steps", type=int, default=20)
    ap.add_argument("--cpu-fstar-sites", type=int, default=1 << 23, help="sites of the CPU f*_M solves (the whole field)")
    ap.add_argument("--cpu-mlp-sites", type=int, default=1 << 16, help="sites of the CPU network-start solve")
    ap.add_argument("--no-fstar", action="store_true", help="skip the f*_M / MLP leg")
    ap.add_argument("--no-active", action="store_true", help="skip the leg with many sites above delta")
    ap.add_argument("--active-rows", type=int, default=256)
    ap.add_argument("--active-steps", type=int, default=192)
    ap.add_argument("--no-cylinder", action="store_true", help="skip the f*_M cylinder run")
    ap.add_argument("--no-wide", action="store_true", help="skip the wide-distribution f*_M solves")
    ap.add_argument("--no-channel", action="store_true", help="skip the 1200 x 400 cylinder channel runs")
    ap.add_argument("--channel-steps", type=int, default=50000)
    ap.add_argument("--cyl-steps", type=int, default=50000)
    ap.add_argument("--fx", type=int, default=4096)
    ap.add_argument("--fy", type=int, default=2048)
    ap.add_argument("--pairs-log2", type=int, default=24)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB float32 tensor 10 times (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the lattice would be split into y-slabs of whole rows with a one-row halo exchange "
              "and an all-gather of the local top-k keys)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0705_4371_amd.lbm as lbm
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain device copy of known size: 2^28 floats (1 GiB) read and written
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 10
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                          "copy_GBps": 2 * (1 << 30) / dt / 1e9}), flush=True)
        return
    prec = lbm.LBM_FP64 if args.precision == "fp64" else lbm.LBM_FP32
    d, rho, u = W.shear_layer(nx=args.nx, ny=args.ny)
    workload = "shear_%dx%d" % (args.nx, args.ny)
    print("# workload %s %s: building fields" % (workload, args.precision), file=sys.stderr, flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        cfg = lbm.config_from_workload(d, prec, stream=stream.cuda_stream)
        lat = lbm.Lattice(cfg, rho, u)
    del rho, u
    n_sites = args.nx * args.ny

    print("# warmup %d" % args.warmup, file=sys.stderr, flush=True)
    lat.step(args.warmup)
    torch.cuda.synchronize()
    settle(lat, torch, args.settle_s)
    # the roofline: K directly launched steps with HIP events around every
    # step kernel on the context's stream
    print("# event-timed %d steps" % args.steps, file=sys.stderr, flush=True)
    dt_ev, k_ms, k_n = timed_steps(lat, torch, args.steps)
    # the headline: K steps as the library runs them by default (replays of
    # the captured 32-step graphs, no events), bracketed by synchronisations
    print("# timed %d steps" % args.steps, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    st, _, _ = lat.stats()
    ms_per_step = dt * 1e3 / args.steps
    mlups = n_sites * args.steps / dt / 1e6
    bytes_per_site = 72 if prec == lbm.LBM_FP32 else 144
    k_avg_ms = k_ms / max(k_n, 1)
    achieved = bytes_per_site * n_sites / (k_avg_ms / 1e3) / 1e9
    # the step kernel is one part of every step, timed or replayed
    assert k_n == args.steps and k_ms <= dt_ev * 1e3 and k_avg_ms <= ms_per_step, \
        ("inconsistent timing", k_avg_ms, dt_ev * 1e3 / args.steps, ms_per_step)
    traffic = traffic_from_profile(workload, args.precision, n_sites)

    out = {
        "metric": "MLUPS + %HBM roofline; MLP-warm vs plain Newton f*_M at <=1e-10 residual",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == lbm.LBM_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": "D2Q9 double shear layer %dx%d periodic, polynomial QE, nu=1e-6, "
                               "delta=1e-4, k=4096" % (args.nx, args.ny),
                   "sites": n_sites, "precision": args.precision},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_step", "kernel_ms": round(k_avg_ms, 4),
                     "kernel_launches": k_n, "bytes_per_site": bytes_per_site,
                     "timing": "HIP events on the context's stream around the k_step of each of the "
                               "%d event-timed steps" % k_n},
        "ehrenfest": {"n_above_delta_last": st.n_above_delta, "selected_total": st.total_selected,
                      "mass": st.mass},
        "settle_s": args.settle_s,
        "timing": "value: the K steps replayed from the library's captured 32-step graphs (its default "
                  "execution); roofline: a preceding pass of K directly launched steps with HIP events "
                  "around each step kernel (event_timed)",
        "event_timed": {"steps": args.steps, "MLUPS": round(n_sites * args.steps / dt_ev / 1e6, 1),
                        "ms_per_step": round(dt_ev * 1e3 / args.steps, 4)},
    }
    if not args.no_active:
        print("# Ehrenfests' steps at full load", file=sys.stderr, flush=True)
        out["ehrenfest_active"] = active_leg(args, torch, lbm, lat, n_sites)
    lat.close()
    if not args.no_fp64 and prec == lbm.LBM_FP32:
        print("# fp64 shear layer", file=sys.stderr, flush=True)
        out["fp64"] = fp64_leg(args, torch, lbm, W)
    if not args.no_channel:
        out["channel_1200x400"] = channel_leg(args, torch, lbm, W)
    net_params = None
    if not args.no_fstar:
        print("# f*_M leg", file=sys.stderr, flush=True)
        out["fstar"], net_params = fstar_leg(args, torch, lbm, W)
    if not args.no_cpu_baseline:
        print("# cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args, net_params)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
