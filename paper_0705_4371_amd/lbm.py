"""Thin Python binding of the C ABI in include/lbm.h.

Argument marshalling only: every step of the method runs in the gfx950
kernels of ``liblbm.so``.  PyTorch provides device memory and the stream.
The functions keep the C names; ``Lattice`` is a small convenience wrapper
that owns a context.  If ``liblbm.so`` is missing the import of this module
raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import _build

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_NONFINITE, LBM_E_NOCONV, LBM_E_STATE = \
    0, -1, -2, -3, -4, -5, -6
LBM_D1Q3, LBM_D2Q9 = 3, 9
LBM_QE_POLY, LBM_QE_ENTROPIC_MM, LBM_QE_ENTROPIC_M = 0, 1, 2
LBM_FP32, LBM_FP64 = 0, 1
LBM_BC_PERIODIC, LBM_BC_ZEROGRAD, LBM_BC_FREESLIP, LBM_BC_INLET_EQ, LBM_BC_OUTLET_EQ, LBM_BC_OUTLET_EQ_PREV = \
    0, 1, 2, 3, 4, 5
LBM_COLL_LBGK, LBM_COLL_ELBM = 0, 1
LBM_START_DEFAULT, LBM_START_CLOSED_FORM, LBM_START_MLP, LBM_START_PREV, LBM_START_PLAIN = 0, 1, 2, 3, 4
LBM_SELECT_AUTO, LBM_SELECT_ONE, LBM_SELECT_MANY = 0, 1, 2


class lbm_config(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("qe", C.c_int32), ("precision", C.c_int32), ("collision", C.c_int32),
        ("nx", C.c_int64), ("ny", C.c_int64),
        ("nu", C.c_double), ("delta", C.c_double),
        ("k", C.c_int32), ("fstar_start", C.c_int32),
        ("bc", C.c_int32 * 4), ("select_mode", C.c_int32), ("reserved", C.c_int32),
        ("inlet_rho", C.c_double), ("inlet_u", C.c_double * 2),
        ("solid_x0", C.c_int64), ("solid_y0", C.c_int64), ("solid_w", C.c_int64), ("solid_h", C.c_int64),
        ("net", C.c_void_p), ("stream", C.c_void_p),
    ]


class lbm_es_stats(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("n_above_delta", C.c_int64), ("n_selected", C.c_int64),
        ("n_invalid", C.c_int64), ("n_fallback", C.c_int64), ("total_selected", C.c_int64),
        ("nonfinite", C.c_int64), ("newton_updates", C.c_int64), ("n_failed", C.c_int64),
        ("kth_dS", C.c_double), ("max_dS", C.c_double), ("mass", C.c_double),
        ("mom", C.c_double * 2), ("energy", C.c_double), ("max_resid", C.c_double),
    ]


class lbm_solve_stats(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("n_infeasible", C.c_int64), ("n_fallback", C.c_int64), ("n_failed", C.c_int64),
        ("iter_hist", C.c_int64 * 16), ("mean_fp32_iters", C.c_double), ("mean_fp64_iters", C.c_double),
        ("max_resid", C.c_double),
    ]


# name -> (restype, argtypes); the exported symbols of include/lbm.h
_P = C.c_void_p
SIGNATURES = {
    "lbm_config_default": (None, [C.POINTER(lbm_config)]),
    "lbm_validate_config": (C.c_int, [C.POINTER(lbm_config)]),
    "lbm_init": (C.c_int, [C.POINTER(lbm_config), _P, _P, _P, C.POINTER(_P)]),
    "lbm_step": (C.c_int, [_P, C.c_int64]),
    "lbm_moments": (C.c_int, [_P, _P, _P, _P]),
    "lbm_get_populations": (C.c_int, [_P, _P]),
    "lbm_set_populations": (C.c_int, [_P, _P]),
    "lbm_ehrenfest_stats": (C.c_int, [_P, C.POINTER(lbm_es_stats), _P, _P, C.c_int64]),
    "lbm_candidates": (C.c_int, [_P, _P, _P, C.c_int64, C.POINTER(C.c_int64)]),
    "lbm_set_timing": (C.c_int, [_P, C.c_int]),
    "lbm_set_fstar_tolerance": (C.c_int, [_P, C.c_double, C.c_double, C.c_int32, C.c_int32]),
    "lbm_kernel_time": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "lbm_layout": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "lbm_struct_sizes": (None, [C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "lbm_probe_set": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int64]),
    "lbm_probe_count": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "lbm_probe_read": (C.c_int, [_P, _P, C.c_int64]),
    "lbm_dft_power": (C.c_int, [_P, C.c_int64, _P, C.POINTER(C.c_int64), _P]),
    "lbm_fstar_create": (C.c_int, [C.c_int64, _P, C.POINTER(_P)]),
    "lbm_fstar_set_tolerance": (C.c_int, [_P, C.c_double, C.c_double, C.c_int32, C.c_int32]),
    "lbm_fstar_solve": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int32, _P, _P, _P, C.POINTER(lbm_solve_stats)]),
    "lbm_fstar_free": (None, [_P]),
    "lbm_fstar_solve_static": (C.c_int, [_P, C.c_int64, _P, C.c_int32, _P, C.c_double, C.c_double, C.c_int32,
                                         C.c_int32, _P, _P, C.POINTER(lbm_solve_stats), _P]),
    "lbm_mlp_create": (C.c_int, [C.c_uint64, C.POINTER(_P)]),
    "lbm_mlp_get_params": (C.c_int, [_P, _P]),
    "lbm_mlp_set_params": (C.c_int, [_P, _P]),
    "lbm_mlp_set_norm": (C.c_int, [_P, _P]),
    "lbm_mlp_get_norm": (C.c_int, [_P, _P]),
    "lbm_mlp_forward": (C.c_int, [_P, _P, C.c_int64, _P, _P]),
    "lbm_mlp_loss_grad": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, _P]),
    "lbm_mlp_adam_step": (C.c_int, [_P, _P, C.c_double, _P]),
    "lbm_mlp_train": (C.c_int, [_P, _P, _P, C.c_int64, C.c_int32, C.c_int32, C.c_double, C.c_uint64, _P, _P]),
    "lbm_mlp_pairs": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, _P]),
    "lbm_mlp_warm_start": (C.c_int, [_P, _P, C.c_int64, _P, _P]),
    "lbm_mlp_free": (None, [_P]),
    "lbm_free": (None, [_P]),
    "lbm_strerror": (C.c_char_p, [C.c_int]),
    "lbm_last_error": (C.c_char_p, []),
}

_lib = None


def load() -> C.CDLL:
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError("liblbm.so is not built (run __graft_entry__.build()); "
                               "there is no CPU fallback for the GPU path")
        # torch first: the library then binds to the HIP runtime that torch
        # loads (torch provides the device memory and streams)
        import torch  # noqa: F401
        L = C.CDLL(_build.LIB)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        a, b = C.c_int64(), C.c_int64()
        L.lbm_struct_sizes(C.byref(a), C.byref(b))
        if (a.value, b.value) != (C.sizeof(lbm_config), C.sizeof(lbm_es_stats)):
            raise RuntimeError("struct layout mismatch between lbm.h and the binding")
        _lib = L
    return _lib


class LbmError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = load()
        msg = L.lbm_last_error().decode(errors="replace")
        super().__init__("%s: %s (%d): %s" % (where, L.lbm_strerror(code).decode(), code, msg))
        self.code = code


def check(code: int, where: str) -> None:
    if code != LBM_OK:
        raise LbmError(code, where)


def make_config(lattice=LBM_D2Q9, qe=LBM_QE_POLY, precision=LBM_FP32, nx=64, ny=64, nu=1e-3,
                delta=math.inf, k=0, bc=(LBM_BC_PERIODIC,) * 4, inlet_rho=1.0, inlet_u=(0.0, 0.0),
                solid=(0, 0, 0, 0), collision=LBM_COLL_LBGK, fstar_start=LBM_START_DEFAULT,
                select_mode=0, stream=None) -> lbm_config:
    c = lbm_config()
    load().lbm_config_default(C.byref(c))
    c.lattice, c.qe, c.precision, c.collision = lattice, qe, precision, collision
    c.nx, c.ny, c.nu, c.delta, c.k = nx, ny, nu, delta, k
    for i in range(4):
        c.bc[i] = bc[i]
    c.inlet_rho = inlet_rho
    c.inlet_u[0], c.inlet_u[1] = inlet_u
    c.solid_x0, c.solid_y0, c.solid_w, c.solid_h = solid
    c.fstar_start = fstar_start
    c.select_mode = select_mode
    c.stream = stream
    return c


def config_from_workload(d: dict, precision: int, stream=None, fstar_start=LBM_START_DEFAULT,
                         net=None, select_mode=0) -> lbm_config:
    """Config from a workloads.* parameter dict (keys Q, qe, nx, ny, nu, ...)."""
    c = make_config(lattice=d["Q"], qe=d.get("qe", LBM_QE_POLY), precision=precision,
                    nx=d["nx"], ny=d["ny"], nu=d["nu"], delta=d.get("delta", math.inf),
                    k=d.get("k", 0), bc=d.get("bc", (LBM_BC_PERIODIC,) * 4),
                    inlet_rho=d.get("inlet_rho", 1.0), inlet_u=d.get("inlet_u", (0.0, 0.0)),
                    solid=d.get("solid", (0, 0, 0, 0)), fstar_start=fstar_start,
                    collision=d.get("collision", LBM_COLL_LBGK), select_mode=select_mode, stream=stream)
    if net is not None:
        c.net = net.h
    return c


class Lattice:
    """Owns one lbm_ctx.  Tensors are torch CUDA tensors; host results numpy."""

    def __init__(self, cfg: lbm_config, rho0, u0, twoE0=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.Q = cfg.lattice
        self.dtype = torch.float64 if cfg.precision == LBM_FP64 else torch.float32
        self.dev = torch.device("cuda", torch.cuda.current_device())
        if cfg.stream is None:
            cfg.stream = torch.cuda.current_stream().cuda_stream
        self.stream_handle = cfg.stream
        r = torch.as_tensor(np.ascontiguousarray(rho0, np.float64), device=self.dev)
        u = torch.as_tensor(np.ascontiguousarray(u0, np.float64), device=self.dev)
        e = None if twoE0 is None else torch.as_tensor(np.ascontiguousarray(twoE0, np.float64),
                                                       device=self.dev)
        ctx = C.c_void_p()
        check(load().lbm_init(C.byref(cfg), r.data_ptr(), u.data_ptr(),
                              e.data_ptr() if e is not None else None, C.byref(ctx)), "lbm_init")
        self.ctx = ctx
        torch.cuda.synchronize()  # the initial fields may be released after this

    def close(self):
        if getattr(self, "ctx", None):
            load().lbm_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.Q, self.cfg.ny, self.cfg.nx)

    def step(self, n: int = 1) -> None:
        check(load().lbm_step(self.ctx, n), "lbm_step")

    def get_populations(self):
        t = self.torch.empty(self.shape, dtype=self.dtype, device=self.dev)
        check(load().lbm_get_populations(self.ctx, t.data_ptr()), "lbm_get_populations")
        return t

    def set_populations(self, f) -> None:
        t = self.torch.as_tensor(f, dtype=self.dtype, device=self.dev).contiguous()
        assert tuple(t.shape) == self.shape
        check(load().lbm_set_populations(self.ctx, t.data_ptr()), "lbm_set_populations")

    def moments(self):
        ny, nx = self.cfg.ny, self.cfg.nx
        rho = self.torch.empty((ny, nx), dtype=self.torch.float64, device=self.dev)
        ru = self.torch.empty((2, ny, nx), dtype=self.torch.float64, device=self.dev)
        e2 = self.torch.empty((ny, nx), dtype=self.torch.float64, device=self.dev)
        check(load().lbm_moments(self.ctx, rho.data_ptr(), ru.data_ptr(), e2.data_ptr()), "lbm_moments")
        return rho, ru, e2

    def stats(self, sel_cap: int = 0):
        st = lbm_es_stats()
        sel = np.zeros(max(sel_cap, 1), np.int64)
        ds = np.zeros(max(sel_cap, 1), np.float64)
        check(load().lbm_ehrenfest_stats(self.ctx, C.byref(st), sel.ctypes.data, ds.ctypes.data,
                                         sel_cap), "lbm_ehrenfest_stats")
        n = min(sel_cap, st.n_selected)
        return st, sel[:n], ds[:n]

    def candidates(self):
        n = C.c_int64()
        check(load().lbm_candidates(self.ctx, None, None, 0, C.byref(n)), "lbm_candidates")
        sites = np.zeros(max(n.value, 1), np.int64)
        ds = np.zeros(max(n.value, 1), np.float64)
        check(load().lbm_candidates(self.ctx, sites.ctypes.data, ds.ctypes.data, n.value, C.byref(n)),
              "lbm_candidates")
        return sites[:n.value], ds[:n.value]

    def set_fstar_tolerance(self, tol: float = None, tol32: float = 2e-6, max32: int = 16,
                            max64: int = 6) -> None:
        """Residual targets and first-pass update budgets of the f*_M solve
        (tol defaults to the context's own: 1e-10 FP32, 1e-13 FP64)."""
        if tol is None:
            tol = 1e-13 if self.cfg.precision == LBM_FP64 else 1e-10
        check(load().lbm_set_fstar_tolerance(self.ctx, tol, tol32, max32, max64), "lbm_set_fstar_tolerance")

    def set_timing(self, on: bool) -> None:
        check(load().lbm_set_timing(self.ctx, int(on)), "lbm_set_timing")

    def kernel_time(self):
        ms = C.c_double()
        n = C.c_int64()
        check(load().lbm_kernel_time(self.ctx, C.byref(ms), C.byref(n)), "lbm_kernel_time")
        return ms.value, n.value

    def layout(self):
        p = C.c_int64()
        b = C.c_int64()
        check(load().lbm_layout(self.ctx, C.byref(p), C.byref(b)), "lbm_layout")
        return p.value, b.value

    def set_probe(self, x: int, y: int, capacity: int) -> None:
        check(load().lbm_probe_set(self.ctx, x, y, capacity), "lbm_probe_set")

    def probe_count(self) -> int:
        n = C.c_int64()
        check(load().lbm_probe_count(self.ctx, C.byref(n)), "lbm_probe_count")
        return n.value

    def probe_read(self, n: int):
        """The last n probe samples, oldest first: cuda float64 [3][n] (rho, u1, u2)."""
        t = self.torch.empty((3, n), dtype=self.torch.float64, device=self.dev)
        check(load().lbm_probe_read(self.ctx, t.data_ptr(), n), "lbm_probe_read")
        return t


def _stream(stream):
    import torch
    return torch.cuda.current_stream().cuda_stream if stream is None else stream


def dft_power(x, stream=None):
    """|DFT|^2 of a real cuda float64 signal at bins 0..n/2 and the dominant
    bin k >= 1 (lbm_dft_power)."""
    import torch
    assert x.dtype == torch.float64 and x.is_cuda and x.dim() == 1
    x = x.contiguous()
    power = torch.empty(x.numel() // 2 + 1, dtype=torch.float64, device=x.device)
    peak = C.c_int64()
    check(load().lbm_dft_power(x.data_ptr(), x.numel(), power.data_ptr(), C.byref(peak), _stream(stream)),
          "lbm_dft_power")
    return power, peak.value


def strouhal(d: dict, rho0, u0, meta: dict, precision: int = LBM_FP32, steps=None, chunk: int = 2000,
             progress=None) -> dict:
    """Shedding frequency of the square-cylinder channel (Sec. 4.2): run
    `steps` (default meta["t_max"] = 1250 L / u_inf) time steps recording u1
    at the monitoring point, take the dominant DFT bin k of the final
    meta["window"] (a quarter) of the n recorded samples, St = L (k / n) / u_inf.
    Stops early, with st = None, when the populations become non-finite
    (checked every `chunk` steps; progress(step, t_max, stats) is called then;
    last_finite_step is the step number of the state kept by the library)."""
    t_max = int(steps if steps is not None else meta["t_max"])
    n = max(2, int(round(meta["window"] * t_max)))
    # one-workgroup selection: a healthy run has few sites above delta, and
    # the run stops at the first chunk with non-finite populations
    lat = Lattice(config_from_workload(d, precision, select_mode=LBM_SELECT_ONE), rho0, u0)
    try:
        lat.set_probe(meta["probe"][0], meta["probe"][1], n)
        done, finite = 0, True
        while done < t_max:
            m = min(chunk, t_max - done)
            lat.step(m)
            done += m
            st, _, _ = lat.stats()
            if st.nonfinite:
                finite = False
                break
            if progress:
                progress(done, t_max, st)
        # after a non-finite step the library keeps the last finite state,
        # whose step number the statistics report
        res = dict(steps=done, finite=finite, last_finite_step=st.step, n=n, st=None, peak=None, series=None)
        if finite:
            series = lat.probe_read(n)
            _, peak = dft_power(series[1])
            res.update(peak=peak, st=meta["L"] * (peak / n) / meta["u_inf"], series=series)
        return res
    finally:
        lat.close()


class FstarSolver:
    """Workspace of the f*_M solver (lbm_fstar_*)."""

    def __init__(self, max_n: int, stream=None):
        import torch
        self.torch = torch
        self.stream = _stream(stream)
        h = C.c_void_p()
        check(load().lbm_fstar_create(max_n, self.stream, C.byref(h)), "lbm_fstar_create")
        self.h = h
        self.max_n = max_n

    def set_tolerance(self, tol=1e-10, tol32=2e-6, max32=16, max64=6):
        check(load().lbm_fstar_set_tolerance(self.h, tol, tol32, max32, max64), "lbm_fstar_set_tolerance")

    def solve(self, M, start=LBM_START_DEFAULT, net=None, stats=True, mu=None, iters=None, status=None):
        """M: cuda float64 [4][n].  Returns (mu, iters, status, stats-or-None)."""
        torch = self.torch
        assert M.dtype == torch.float64 and M.is_cuda and M.dim() == 2 and M.shape[0] == 4
        M = M.contiguous()
        n = M.shape[1]
        if mu is None:
            mu = torch.empty_like(M)
        if iters is None:
            iters = torch.empty(n, dtype=torch.uint8, device=M.device)
        if status is None:
            status = torch.empty(n, dtype=torch.uint8, device=M.device)
        st = lbm_solve_stats() if stats else None
        rc = load().lbm_fstar_solve(self.h, M.data_ptr(), n, mu.data_ptr(), start,
                                    net.h if net is not None else None, iters.data_ptr(),
                                    status.data_ptr(), C.byref(st) if st is not None else None)
        if rc not in (LBM_OK, LBM_E_NOCONV):
            check(rc, "lbm_fstar_solve")
        return mu, iters, status, st

    def close(self):
        if getattr(self, "h", None):
            load().lbm_fstar_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


LBM_FSTAR_STATIC_MLP_MAX = 1 << 20
LBM_FSTAR_STATIC_MAX_N = 1 << 23


def fstar_solve_static(M, start=LBM_START_DEFAULT, net=None, stats=True, mu=None, iters=None, status=None,
                       tol=1e-10, tol32=2e-6, max32=16, max64=6, stream=None):
    """lbm_fstar_solve_static (no solver handle, no allocation in the
    library).  M: cuda float64 [4][n].  Returns (mu, iters, status,
    stats-or-None)."""
    import torch
    assert M.dtype == torch.float64 and M.is_cuda and M.dim() == 2 and M.shape[0] == 4
    M = M.contiguous()
    n = M.shape[1]
    if mu is None:
        mu = torch.empty_like(M)
    if iters is None:
        iters = torch.empty(n, dtype=torch.uint8, device=M.device)
    if status is None:
        status = torch.empty(n, dtype=torch.uint8, device=M.device)
    st = lbm_solve_stats() if stats else None
    rc = load().lbm_fstar_solve_static(M.data_ptr(), n, mu.data_ptr(), start, net.h if net is not None else None,
                                       tol, tol32, max32, max64, iters.data_ptr(), status.data_ptr(),
                                       C.byref(st) if st is not None else None, _stream(stream))
    if rc not in (LBM_OK, LBM_E_NOCONV):
        check(rc, "lbm_fstar_solve_static")
    return mu, iters, status, st


class Mlp:
    """The warm-start network (lbm_mlp_*)."""

    NPARAM = 4740

    def __init__(self, seed: int = 0):
        import torch
        self.torch = torch
        h = C.c_void_p()
        check(load().lbm_mlp_create(seed, C.byref(h)), "lbm_mlp_create")
        self.h = h

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.NPARAM, np.float32)
        check(load().lbm_mlp_get_params(self.h, p.ctypes.data), "lbm_mlp_get_params")
        return p

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == self.NPARAM
        check(load().lbm_mlp_set_params(self.h, p.ctypes.data), "lbm_mlp_set_params")

    def set_norm(self, in_shift, in_scale, out_shift, out_scale) -> None:
        v = np.ascontiguousarray(np.concatenate([in_shift, in_scale, out_shift, out_scale]), np.float32)
        check(load().lbm_mlp_set_norm(self.h, v.ctypes.data), "lbm_mlp_set_norm")

    def get_norm(self) -> np.ndarray:
        v = np.zeros(16, np.float32)
        check(load().lbm_mlp_get_norm(self.h, v.ctypes.data), "lbm_mlp_get_norm")
        return v

    def forward(self, X, stream=None):
        X = X.contiguous()
        Y = self.torch.empty_like(X)
        check(load().lbm_mlp_forward(self.h, X.data_ptr(), X.shape[0], Y.data_ptr(), _stream(stream)),
              "lbm_mlp_forward")
        return Y

    def loss_grad(self, X, T, stream=None):
        torch = self.torch
        g = torch.empty(self.NPARAM, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        check(load().lbm_mlp_loss_grad(self.h, X.contiguous().data_ptr(), T.contiguous().data_ptr(), X.shape[0],
                                       g.data_ptr(), loss.data_ptr(), _stream(stream)), "lbm_mlp_loss_grad")
        return loss, g

    def adam_step(self, grad, lr=1e-3, stream=None):
        check(load().lbm_mlp_adam_step(self.h, grad.data_ptr(), lr, _stream(stream)), "lbm_mlp_adam_step")

    def pairs(self, M, mu=None, stream=None):
        """Normalised network inputs X [n][4] of moments M (cuda float64
        [4][n]) and, with multipliers mu [4][n], targets T [n][4]
        (lbm_mlp_pairs).  Returns (X, T or None)."""
        torch = self.torch
        M = M.contiguous()
        n = M.shape[1]
        X = torch.empty((n, 4), dtype=torch.float32, device=M.device)
        T = torch.empty((n, 4), dtype=torch.float32, device=M.device) if mu is not None else None
        check(load().lbm_mlp_pairs(self.h, M.data_ptr(), mu.contiguous().data_ptr() if mu is not None else None, n,
                                   X.data_ptr(), T.data_ptr() if T is not None else None, _stream(stream)),
              "lbm_mlp_pairs")
        return X, T

    def warm_start(self, M, out=None, stream=None):
        """The solver's network start (mu0 - ln rho, mu1, mu2, mu3) [4][n]
        (float32; into out when given) for moments M (float64 [4][n] on the
        device) (lbm_mlp_warm_start)."""
        M = M.contiguous()
        n = M.shape[1]
        warm = out if out is not None else self.torch.empty((4, n), dtype=self.torch.float32, device=M.device)
        assert warm.shape == (4, n) and warm.dtype == self.torch.float32 and warm.is_contiguous()
        check(load().lbm_mlp_warm_start(self.h, M.data_ptr(), n, warm.data_ptr(), _stream(stream)),
              "lbm_mlp_warm_start")
        return warm

    def train(self, X, T, epochs, batch, lr=1e-3, seed=0, stream=None) -> np.ndarray:
        losses = np.zeros(max(epochs, 1), np.float32)
        check(load().lbm_mlp_train(self.h, X.contiguous().data_ptr(), T.contiguous().data_ptr(), X.shape[0],
                                   epochs, batch, lr, seed, losses.ctypes.data, _stream(stream)), "lbm_mlp_train")
        return losses[:epochs]

    def close(self):
        if getattr(self, "h", None):
            load().lbm_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
