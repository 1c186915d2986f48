"""Host-only checks of the C-ABI library (no GPU): it loads, exports every
function declared in include/lbm.h, its struct layouts match the binding,
and invalid configurations are rejected before any HIP call."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_0705_4371_amd import _build
    if _build.stale():
        _build.build()
    import paper_0705_4371_amd.lbm as lbm
    return lbm


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(lbm_[a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert len(names) >= 15
    lib = C.CDLL(os.path.join(ROOT, "paper_0705_4371_amd", "liblbm.so"))
    for n in names:
        assert hasattr(lib, n), n
    # and the binding covers all of them
    assert set(names) <= set(L.SIGNATURES), set(names) - set(L.SIGNATURES)


def test_struct_layout(L):
    L.load()  # raises on mismatch


def test_strerror(L):
    lib = L.load()
    assert lib.lbm_strerror(L.LBM_E_INVAL) == b"invalid argument"
    assert lib.lbm_strerror(0) == b"ok"


def _bad(L, **kw):
    cfg = L.make_config(**kw)
    rc = L.load().lbm_validate_config(C.byref(cfg))
    return rc, L.load().lbm_last_error().decode()


@pytest.mark.parametrize("kw,frag", [
    (dict(lattice=5), "lattice"),
    (dict(qe=7), "qe"),
    (dict(precision=3), "precision"),
    (dict(nx=1), "nx >= 2"),
    (dict(lattice=3, ny=4), "D1Q3"),
    (dict(nu=-1.0), "nu"),
    (dict(nu=math.nan), "nu"),
    (dict(delta=-1e-3), "delta"),
    (dict(k=-2), "k must"),
    (dict(bc=(1, 0, 0, 0)), "west and east"),
    (dict(bc=(0, 0, 3, 3)), "not allowed"),
    (dict(bc=(2, 2, 0, 0)), "not allowed"),
    (dict(solid=(60, 60, 10, 10)), "inside"),
    (dict(bc=(3, 1, 2, 2), inlet_rho=0.0), "inlet"),
    (dict(nx=70000, ny=70000), "too large"),
    (dict(nx=(1 << 25) + 1, ny=1, lattice=3), "too large"),
    (dict(collision=1), "ELBM needs"),
    (dict(collision=4, qe=1), "collision"),
    (dict(qe=2, lattice=3, ny=1), "D2Q9"),
    (dict(qe=2, fstar_start=4), "fstar_start"),
    (dict(bc=(0, 0, 4, 4)), "not allowed"),
    (dict(select_mode=3), "select_mode"),
    (dict(nx=2, ny=4, bc=(3, 4, 2, 2)), "nx >= 3"),
    (dict(nx=100, ny=50, bc=(3, 4, 2, 2), solid=(60, 20, 39, 5)), "clear of an outlet"),
    (dict(nx=100, ny=50, bc=(4, 3, 2, 2), solid=(1, 20, 10, 5)), "clear of an outlet"),
])
def test_invalid_configs_rejected(L, kw, frag):
    rc, msg = _bad(L, **kw)
    assert rc == L.LBM_E_INVAL and frag in msg, (rc, msg)


def test_valid_configs_accepted(L):
    for kw in (dict(), dict(lattice=3, nx=800, ny=1, bc=(1, 1, 0, 0), delta=1e-3, k=4, precision=1),
               dict(nx=1200, ny=400, bc=(3, 1, 2, 2), inlet_u=(0.05, 0.0), solid=(280, 180, 40, 40),
                    delta=1e-3, k=64),
               dict(nx=600, ny=500, qe=1, bc=(3, 4, 2, 2), inlet_u=(0.05, 0.0), solid=(200, 240, 20, 20),
                    delta=1e-3, k=10),
               dict(nx=100, ny=50, bc=(3, 4, 2, 2), solid=(60, 20, 38, 5)),
               dict(lattice=3, nx=3, ny=1, bc=(3, 4, 0, 0))):
        rc, msg = _bad(L, **kw)
        assert rc == 0, msg


def test_init_rejects_null_arguments_without_gpu(L):
    cfg = L.make_config()
    out = C.c_void_p()
    assert L.load().lbm_init(C.byref(cfg), None, None, None, C.byref(out)) == L.LBM_E_INVAL
    assert L.load().lbm_step(None, 1) == L.LBM_E_INVAL


def test_probe_and_spectrum_reject_bad_arguments_without_gpu(L):
    lib = L.load()
    n = C.c_int64()
    assert lib.lbm_probe_set(None, 0, 0, 10) == L.LBM_E_INVAL
    assert lib.lbm_probe_count(None, C.byref(n)) == L.LBM_E_INVAL
    assert lib.lbm_probe_read(None, None, 1) == L.LBM_E_INVAL
    buf = (C.c_double * 4)()
    assert lib.lbm_dft_power(None, 4, buf, None, None) == L.LBM_E_INVAL
    assert lib.lbm_dft_power(buf, 0, buf, None, None) == L.LBM_E_INVAL
    assert lib.lbm_dft_power(buf, (1 << 31) + 1, buf, None, None) == L.LBM_E_INVAL
    assert lib.lbm_set_fstar_tolerance(None, 1e-10, 2e-6, 16, 6) == L.LBM_E_INVAL


def test_learned_start_entries_reject_bad_arguments_without_gpu(L):
    """The network's pairs and start entries and the allocation-free solve
    validate their arguments on the host, before any HIP call."""
    lib = L.load()
    buf = (C.c_double * 8)()
    out = (C.c_float * 8)()
    assert lib.lbm_mlp_warm_start(None, buf, 1, out, None) == L.LBM_E_INVAL
    assert lib.lbm_mlp_warm_start(None, buf, -1, out, None) == L.LBM_E_INVAL
    assert lib.lbm_mlp_pairs(None, buf, None, 1, out, None, None) == L.LBM_E_INVAL
    # a start outside LBM_START_* is refused before the solve touches a device
    assert lib.lbm_fstar_solve_static(buf, 1, buf, 7, None, 1e-10, 2e-6, 16, 6, None, None, None, None) \
        == L.LBM_E_INVAL
