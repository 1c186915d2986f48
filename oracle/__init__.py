"""Plain FP64 CPU oracle for the Ehrenfests'-step-regularised lattice
Boltzmann method (Brownlee, Gorban, Levesley 2007) and for the learned warm
start of its entropic quasiequilibrium solve.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  It shares no code with
the GPU library ``paper_0705_4371_amd``; all of its arithmetic lives in
``oracle.c`` (plain C, FP64, long double for Delta S); this module only
marshals numpy arrays and composes those functions.

Every function names the passage of the paper it follows in ``oracle.c``.
Functions without an independent pin are listed as "parity unpinned" in the
design notes; every function here has at least one pin in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source built with OpenMP over its site loops: for timing only
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

QE_POLY, QE_ENTROPIC_MM, QE_ENTROPIC_M = 0, 1, 2
BC_PERIODIC, BC_ZEROGRAD, BC_FREESLIP, BC_INLET_EQ, BC_OUTLET_EQ, BC_OUTLET_EQ_PREV = 0, 1, 2, 3, 4, 5
COLL_LBGK, COLL_ELBM = 0, 1
MLP_NPARAM = 4740


def build(force: bool = True, omp: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, no fast-math,
    single-threaded: the parity reference); with omp=True into liboracle_omp.so with
    OpenMP over the site loops (the same arithmetic per site; used only to
    time the oracle on all host cores)."""
    out = _LIB_OMP if omp else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
             "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"] + (["-fopenmp"] if omp else []) + [_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


class _Cfg(C.Structure):
    _fields_ = [
        ("Q", C.c_int32), ("qe", C.c_int32), ("collision", C.c_int32), ("pad0", C.c_int32),
        ("nx", C.c_int64), ("ny", C.c_int64),
        ("nu", C.c_double), ("delta", C.c_double), ("k", C.c_int64),
        ("bc", C.c_int32 * 4),
        ("inlet_rho", C.c_double), ("inlet_u1", C.c_double), ("inlet_u2", C.c_double),
        ("solid_x0", C.c_int64), ("solid_y0", C.c_int64), ("solid_w", C.c_int64), ("solid_h", C.c_int64),
    ]


class _Info(C.Structure):
    _fields_ = [("n_above", C.c_int64), ("n_selected", C.c_int64), ("n_invalid", C.c_int64),
                ("n_fallback", C.c_int64), ("sums", C.c_double * 4)]


_lib = None
_lib_omp = None
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_I32 = C.POINTER(C.c_int32)
_F32 = C.POINTER(C.c_float)


def lib(omp: bool = False):
    """The plain oracle library, or (omp=True) its OpenMP timing build."""
    global _lib, _lib_omp
    if omp:
        if _lib_omp is None:
            if not os.path.exists(_LIB_OMP) or os.path.getmtime(_LIB_OMP) < os.path.getmtime(_SRC):
                build(force=True, omp=True)
            _lib_omp = _declare(C.CDLL(_LIB_OMP))
        return _lib_omp
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _declare(C.CDLL(_LIB))
    return _lib


def _declare(L):
    """Argument and result types of the exported functions."""
    L.or_velocities.argtypes = [C.c_int, _I32, _I32, _D]
    L.or_moments.argtypes = [C.c_int, _D, _D]
    L.or_qe_poly.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _D]
    L.or_qe_entropic_mm.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _D]
    L.or_fstar_feasible.argtypes = [_D]
    L.or_fstar_newton.argtypes = [_D, C.c_double, C.c_int, _D, _D]
    L.or_fstar_scalar.argtypes = [_D, _D]
    L.or_fstar_polish.argtypes = [_D, _D]
    L.or_fstar_polish.restype = C.c_double
    L.or_fstar_from_mu.argtypes = [_D, _D]
    L.or_dft_power.argtypes = [_D, C.c_int64, _D]
    L.or_dft_power.restype = None
    L.or_dft_power_at.argtypes = [_D, C.c_int64, C.c_int64]
    L.or_dft_power_at.restype = C.c_double
    L.or_delta_S.argtypes = [C.c_int, _D, _D]
    L.or_delta_S.restype = C.c_longdouble
    L.or_elbm_alpha.argtypes = [C.c_int, _D, _D]
    L.or_elbm_alpha.restype = C.c_double
    L.or_elbm_H.argtypes = [C.c_int, _D, _D, C.c_longdouble]
    L.or_elbm_H.restype = C.c_longdouble
    L.or_init.argtypes = [C.POINTER(_Cfg), _D, _D, _D, _D]
    L.or_step.argtypes = [C.POINTER(_Cfg), _D, _D, _D, _I64, C.POINTER(_Info)]
    L.or_step_sites.argtypes = [C.POINTER(_Cfg), _D, _I64, C.c_int64, _I64, C.c_int64, _D]
    L.or_site_dS.argtypes = [C.POINTER(_Cfg), _D, C.c_int64]
    L.or_site_dS.restype = C.c_double
    L.or_sums.argtypes = [C.POINTER(_Cfg), _D, _D]
    L.or_sums.restype = None
    L.or_mlp_forward.argtypes = [_D, _D, C.c_int64, _D, C.c_int]
    L.or_mlp_forward.restype = C.c_double
    L.or_mlp_loss_grad.argtypes = [_D, _D, _D, C.c_int64, _D, C.c_int]
    L.or_mlp_loss_grad.restype = C.c_double
    L.or_adam_step.argtypes = [_D, _D, _D, _D, C.c_int64, C.c_int64, C.c_double, C.c_double,
                               C.c_double, C.c_double]
    L.or_bf16_round.argtypes = [C.c_double]
    L.or_bf16_round.restype = C.c_double
    L.or_mlp_features.argtypes = [_D, C.c_int64, _F32, _D]
    L.or_mlp_features.restype = None
    L.or_mlp_targets.argtypes = [_D, _D, C.c_int64, _F32, _D]
    L.or_mlp_targets.restype = None
    L.or_mlp_unnormalise.argtypes = [_D, C.c_int64, _F32, _D]
    L.or_mlp_unnormalise.restype = None
    L.or_fstar_field.argtypes = [_D, C.c_int64, C.c_double, C.c_int, _D, _I32]
    L.or_fstar_field.restype = C.c_int64
    return L


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def velocities(Q: int):
    vx = np.zeros(Q, np.int32)
    vy = np.zeros(Q, np.int32)
    w = np.zeros(Q, np.float64)
    rc = lib().or_velocities(Q, vx.ctypes.data_as(_I32), vy.ctypes.data_as(_I32), _p(w))
    if rc != 0:
        raise ValueError("Q must be 3 or 9")
    return vx, vy, w


def moments(Q: int, f) -> np.ndarray:
    f = np.ascontiguousarray(f, np.float64)
    M = np.zeros(4)
    lib().or_moments(Q, _p(f), _p(M))
    return M


def qe_poly(Q: int, rho: float, u1: float, u2: float = 0.0) -> np.ndarray:
    out = np.zeros(Q)
    lib().or_qe_poly(Q, rho, u1, u2, _p(out))
    return out


def qe_entropic_mm(Q: int, rho: float, u1: float, u2: float = 0.0) -> np.ndarray:
    out = np.zeros(Q)
    lib().or_qe_entropic_mm(Q, rho, u1, u2, _p(out))
    return out


def fstar_feasible(M) -> bool:
    M = np.ascontiguousarray(M, np.float64)
    return bool(lib().or_fstar_feasible(_p(M)))


def fstar_newton(M, tol: float = 1e-13, max_iter: int = 100):
    """f*_M multipliers by damped Newton.  Returns (mu, iterations, residual);
    iterations < 0 flags an infeasible (-1) or unconverged (-2) site."""
    M = np.ascontiguousarray(M, np.float64)
    mu = np.zeros(4)
    r = np.zeros(1)
    it = lib().or_fstar_newton(_p(M), tol, max_iter, _p(mu), _p(r))
    return mu, int(it), float(r[0])


def fstar_polish(M, mu):
    """One more Newton update of converged multipliers (or_fstar_polish).
    Returns (mu, residual)."""
    M = np.ascontiguousarray(M, np.float64)
    mu = np.array(mu, np.float64)
    r = lib().or_fstar_polish(_p(M), _p(mu))
    return mu, float(r)


def fstar_field(M, tol=1e-10, start=0, mu=None, omp=False):
    """Damped-Newton f*_M of a moment field M [4][n] (or_fstar_field): start
    0 rest, 1 mass-momentum closed form, 2 the multipliers in mu.  Returns
    (mu [4][n], iterations [n] (negative: infeasible / unconverged), number of
    unconverged sites)."""
    M = np.ascontiguousarray(M, np.float64)
    n = M.shape[1]
    mu = np.zeros((4, n)) if mu is None else np.ascontiguousarray(mu, np.float64).copy()
    it = np.zeros(n, np.int32)
    bad = lib(omp).or_fstar_field(_p(M), n, tol, start, _p(mu), it.ctypes.data_as(_I32))
    return mu, it, int(bad)


def fstar_scalar(M):
    """f*_M multipliers through the product structure and bisection on ln Z."""
    M = np.ascontiguousarray(M, np.float64)
    mu = np.zeros(4)
    rc = lib().or_fstar_scalar(_p(M), _p(mu))
    return (mu if rc == 0 else None)


def fstar_from_mu(mu) -> np.ndarray:
    mu = np.ascontiguousarray(mu, np.float64)
    out = np.zeros(9)
    lib().or_fstar_from_mu(_p(mu), _p(out))
    return out


def delta_S(f, fs) -> float:
    f = np.ascontiguousarray(f, np.float64)
    fs = np.ascontiguousarray(fs, np.float64)
    return float(lib().or_delta_S(len(f), _p(f), _p(fs)))


def elbm_alpha(f, fs) -> float:
    f = np.ascontiguousarray(f, np.float64)
    fs = np.ascontiguousarray(fs, np.float64)
    return float(lib().or_elbm_alpha(len(f), _p(f), _p(fs)))


def elbm_H(f, fs, a) -> float:
    """S(f + a (f* - f)) - S(f) in the cancellation-free form (entropic f*)."""
    f = np.ascontiguousarray(f, np.float64)
    fs = np.ascontiguousarray(fs, np.float64)
    return float(lib().or_elbm_H(len(f), _p(f), _p(fs), a))


def make_cfg(Q=9, qe=QE_POLY, nx=16, ny=1, nu=1e-3, delta=float("inf"), k=0,
             bc=(BC_PERIODIC,) * 4, inlet_rho=1.0, inlet_u=(0.0, 0.0), solid=(0, 0, 0, 0),
             collision=COLL_LBGK) -> _Cfg:
    c = _Cfg()
    c.Q, c.qe, c.collision = Q, qe, collision
    c.nx, c.ny = nx, ny
    c.nu, c.delta, c.k = nu, delta, k
    for i in range(4):
        c.bc[i] = bc[i]
    c.inlet_rho, c.inlet_u1, c.inlet_u2 = inlet_rho, inlet_u[0], inlet_u[1]
    c.solid_x0, c.solid_y0, c.solid_w, c.solid_h = solid
    return c


def cfg_from_dict(d: dict) -> _Cfg:
    return make_cfg(**d)


def init(cfg: _Cfg, rho0, u0, twoE0=None) -> np.ndarray:
    """f(x, 0) = quasiequilibrium of (rho0, u0[, 2E0]); arrays [ny][nx], u0 [2][ny][nx]."""
    N = cfg.nx * cfg.ny
    rho0 = np.ascontiguousarray(rho0, np.float64).reshape(-1)
    u0 = np.ascontiguousarray(u0, np.float64).reshape(-1)
    assert rho0.size == N and u0.size in (N, 2 * N)
    if u0.size == N:
        u0 = np.concatenate([u0, np.zeros(N)])
    f = np.zeros((cfg.Q, cfg.ny, cfg.nx))
    e = None
    if twoE0 is not None:
        e = np.ascontiguousarray(twoE0, np.float64).reshape(-1)
    lib().or_init(C.byref(cfg), _p(rho0), _p(u0), _p(e) if e is not None else None, _p(f))
    return f


def step(cfg: _Cfg, f_in: np.ndarray, omp: bool = False) -> dict:
    """One time step (pre-collision f(t) -> pre-collision f(t+1)).  Returns
    dict(f, dS, sel, n_above, n_selected, n_invalid, n_fallback, sums).
    omp=True runs the OpenMP timing build."""
    f_in = np.ascontiguousarray(f_in, np.float64)
    assert f_in.shape == (cfg.Q, cfg.ny, cfg.nx)
    f_out = np.zeros_like(f_in)
    dS = np.zeros((cfg.ny, cfg.nx))
    sel = np.zeros(max(int(cfg.k), 1), np.int64)
    info = _Info()
    rc = lib(omp).or_step(C.byref(cfg), _p(f_in), _p(f_out), _p(dS), sel.ctypes.data_as(_I64),
                          C.byref(info))
    if rc != 0:
        raise MemoryError("oracle step failed (%d)" % rc)
    return dict(f=f_out, dS=dS, sel=sel[:info.n_selected].copy(), n_above=info.n_above,
                n_selected=info.n_selected, n_invalid=info.n_invalid,
                n_fallback=info.n_fallback, sums=np.array(info.sums[:]))


def step_sites(cfg: _Cfg, f_in: np.ndarray, sites, selected) -> np.ndarray:
    """f(t+1) at the given output sites [ns][Q], from f(t) with the given set
    of sites returned to quasiequilibrium (for lattices too large for step)."""
    f_in = np.ascontiguousarray(f_in, np.float64)
    sites = np.ascontiguousarray(sites, np.int64)
    sel = np.ascontiguousarray(np.asarray(selected, np.int64).reshape(-1))
    out = np.zeros((sites.size, cfg.Q))
    lib().or_step_sites(C.byref(cfg), _p(f_in), sites.ctypes.data_as(_I64), sites.size,
                        sel.ctypes.data_as(_I64) if sel.size else None, sel.size, _p(out))
    return out


def site_dS(cfg: _Cfg, f_in: np.ndarray, sites) -> np.ndarray:
    f_in = np.ascontiguousarray(f_in, np.float64)
    return np.array([lib().or_site_dS(C.byref(cfg), _p(f_in), int(s)) for s in np.asarray(sites).reshape(-1)])


def sums(cfg: _Cfg, f: np.ndarray) -> np.ndarray:
    """Sums over the fluid sites of rho, rho u1, rho u2, 2E of a state f
    [Q][ny][nx] (or_sums: long double accumulation)."""
    f = np.ascontiguousarray(f, np.float64)
    assert f.shape == (cfg.Q, cfg.ny, cfg.nx)
    out = np.zeros(4)
    lib().or_sums(C.byref(cfg), _p(f), _p(out))
    return out


def dft_power(x) -> np.ndarray:
    """|DFT|^2 of a real signal at bins 0..n/2, by the definition (or_dft_power);
    the shedding frequency of Sec. 4.2 is the dominant bin of the last quarter
    of the recorded velocity."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1)
    out = np.zeros(x.size // 2 + 1)
    lib().or_dft_power(_p(x), x.size, _p(out))
    return out


def dft_power_at(x, bins) -> np.ndarray:
    """dft_power at the given bins only (O(n) each)."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1)
    return np.array([lib().or_dft_power_at(_p(x), x.size, int(k)) for k in np.asarray(bins).reshape(-1)])


def run(cfg: _Cfg, f: np.ndarray, nsteps: int) -> np.ndarray:
    for _ in range(nsteps):
        f = step(cfg, f)["f"]
    return f


# ---------------------------------------------------------------------------
# MLP 4 -> 64 -> 64 -> 4 (SiLU)
# ---------------------------------------------------------------------------

def bf16_round(x: float) -> float:
    return float(lib().or_bf16_round(float(x)))


def mlp_forward(params, x, bf16: bool = False) -> np.ndarray:
    p = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    n = x.shape[0]
    y = np.zeros((n, 4))
    lib().or_mlp_forward(_p(p), _p(x), n, _p(y), int(bf16))
    return y


def mlp_loss_grad(params, x, t, bf16: bool = False):
    p = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    g = np.zeros(MLP_NPARAM)
    loss = lib().or_mlp_loss_grad(_p(p), _p(x), _p(t), x.shape[0], _p(g), int(bf16))
    return float(loss), g


def adam_step(p, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays p, m, v."""
    lib().or_adam_step(_p(p), _p(m), _p(v), _p(np.ascontiguousarray(g, np.float64)), p.size, t,
                       lr, b1, b2, eps)


# ---------------------------------------------------------------------------
# Learned warm start of the f*_M solve: features, targets, network start
# ---------------------------------------------------------------------------

def _norm(norm16) -> np.ndarray:
    nm = np.ascontiguousarray(np.asarray(norm16, np.float32).reshape(16))
    return nm


def mlp_features(M, norm16) -> np.ndarray:
    """Normalised network inputs [n][4] of moment vectors M [4][n]
    (or_mlp_features: (u1, u2, 2E/rho, |u|^2), shifted and scaled by
    norm16[0:4], norm16[4:8], rounded to FP32)."""
    M = np.ascontiguousarray(M, np.float64)
    n = M.shape[1]
    nm = _norm(norm16)
    X = np.zeros((n, 4))
    lib().or_mlp_features(_p(M), n, nm.ctypes.data_as(_F32), _p(X))
    return X


def mlp_targets(M, mu, norm16) -> np.ndarray:
    """Normalised network targets [n][4] of multipliers mu [4][n]
    (or_mlp_targets: (mu0 - ln rho, mu1, mu2, mu3), shifted and scaled by
    norm16[8:12], norm16[12:16])."""
    M = np.ascontiguousarray(M, np.float64)
    mu = np.ascontiguousarray(mu, np.float64)
    n = M.shape[1]
    nm = _norm(norm16)
    T = np.zeros((n, 4))
    lib().or_mlp_targets(_p(M), _p(mu), n, nm.ctypes.data_as(_F32), _p(T))
    return T


def mlp_unnormalise(Y, norm16) -> np.ndarray:
    """Network outputs Y [n][4] back to (mu0 - ln rho, mu1, mu2, mu3) [4][n]."""
    Y = np.ascontiguousarray(Y, np.float64)
    n = Y.shape[0]
    nm = _norm(norm16)
    out = np.zeros((4, n))
    lib().or_mlp_unnormalise(_p(Y), n, nm.ctypes.data_as(_F32), _p(out))
    return out


def mlp_warm_start(params, norm16, M) -> np.ndarray:
    """Network start (mu0 - ln rho, mu1, mu2, mu3) [4][n] for moments M:
    features, forward pass with the BF16 rounding points of the GPU kernels
    emulated, outputs unnormalised."""
    y = mlp_forward(params, mlp_features(M, norm16), bf16=True)
    return mlp_unnormalise(y, norm16)
