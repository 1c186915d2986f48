"""lbm_fstar_solve_static (the solver entry for callers that cannot allocate)
against lbm_fstar_solve on the same inputs: the same kernels, so
bit-identical multipliers, iteration counts, statuses and statistics, for
every start, with forced fallbacks, on two calls in a row (the second with
fewer sites, so that state left in the shared static scratch by the first
would show)."""
import numpy as np
import pytest

import workloads as W
from _gpu_common import say, torch_gpu

pytestmark = pytest.mark.gpu


def _stats_tuple(st):
    return (st.n, st.n_infeasible, st.n_fallback, st.n_failed, tuple(st.iter_hist), st.mean_fp32_iters,
            st.mean_fp64_iters, st.max_resid)


def _compare(lbm, solver, M, start, net=None, mu0=None, tol=(1e-10, 2e-6, 16, 6), label=""):
    torch = torch_gpu()
    solver.set_tolerance(*tol)
    mu_a = mu0.clone() if mu0 is not None else None
    mu_b = mu0.clone() if mu0 is not None else None
    mu_a, it_a, sa_, st_a = solver.solve(M, start=start, net=net, mu=mu_a)
    mu_b, it_b, sb_, st_b = lbm.fstar_solve_static(M, start=start, net=net, mu=mu_b, tol=tol[0], tol32=tol[1],
                                                   max32=tol[2], max64=tol[3])
    torch.cuda.synchronize()
    say("  %s n=%d fallback %d failed %d" % (label, M.shape[1], st_b.n_fallback, st_b.n_failed))
    assert torch.equal(mu_a, mu_b), label
    assert torch.equal(it_a, it_b) and torch.equal(sa_, sb_), label
    assert _stats_tuple(st_a) == _stats_tuple(st_b), (label, _stats_tuple(st_a), _stats_tuple(st_b))
    return st_b


def test_static_solve_matches_handle_solve():
    torch = torch_gpu()
    import paper_0705_4371_amd.lbm as lbm
    n1, n2 = 1 << 18, (1 << 16) + 123
    M1 = torch.from_numpy(W.random_moments(n1, 6, umax=0.2, energy_band=0.2)).cuda()
    M2 = torch.from_numpy(W.random_moments(n2, 7, umax=0.2, energy_band=0.2)).cuda()
    solver = lbm.FstarSolver(n1)
    net = lbm.Mlp(3)
    ish, isc, osh, _ = W.mlp_norm()
    net.set_norm(ish, isc, osh, [0.05] * 4)  # an untrained network scaled up: a poor start
    say("case static f*_M solve against the handle solve")
    for M in (M1, M2):
        n = M.shape[1]
        _compare(lbm, solver, M, lbm.LBM_START_DEFAULT, label="rest")
        _compare(lbm, solver, M, lbm.LBM_START_CLOSED_FORM, label="closed form")
        _compare(lbm, solver, M, lbm.LBM_START_PLAIN, label="plain FP64 Newton")
        _compare(lbm, solver, M, lbm.LBM_START_MLP, net=net, label="network")
        mu_prev, _, _, _ = solver.solve(M, start=lbm.LBM_START_DEFAULT)
        mu_prev = mu_prev * (1 + 1e-3 * torch.sin(torch.arange(n, device=M.device, dtype=M.dtype)))
        _compare(lbm, solver, M, lbm.LBM_START_PREV, mu0=mu_prev, label="previous")
        # every site through the inline fallback
        st = _compare(lbm, solver, M, lbm.LBM_START_DEFAULT, tol=(1e-13, 2e-6, 0, 1), label="forced fallback")
        assert st.n_fallback >= 0.99 * n and st.n_failed == 0
    solver.close()
    net.close()


def test_static_solve_limits():
    torch = torch_gpu()
    import paper_0705_4371_amd.lbm as lbm
    n = lbm.LBM_FSTAR_STATIC_MLP_MAX + 1
    M = torch.ones((4, n), dtype=torch.float64, device="cuda")
    net = lbm.Mlp(1)
    with pytest.raises(lbm.LbmError) as e:
        lbm.fstar_solve_static(M, start=lbm.LBM_START_MLP, net=net)
    assert e.value.code == lbm.LBM_E_INVAL and "static scratch" in str(e.value)
    # sizes beyond the failure list are rejected on the host (no kernel runs)
    big = torch.ones((4, 1), dtype=torch.float64, device="cuda").expand(4, lbm.LBM_FSTAR_STATIC_MAX_N + 1)
    L = lbm.load()
    rc = L.lbm_fstar_solve_static(big.data_ptr(), lbm.LBM_FSTAR_STATIC_MAX_N + 1, big.data_ptr(), 0, None, 1e-10,
                                  2e-6, 16, 6, None, None, None, None)
    assert rc == lbm.LBM_E_INVAL
    with pytest.raises(lbm.LbmError) as e:
        lbm.fstar_solve_static(M[:, :16], start=lbm.LBM_START_DEFAULT, tol=-1.0)
    assert e.value.code == lbm.LBM_E_INVAL
    net.close()
