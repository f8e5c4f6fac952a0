"""Host-only checks of the C ABI library: it loads, exports every function
include/stokes.h declares, and its host-side sizing/validation agrees with the
documented layout.  No kernel is launched (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1308_4605_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "stokes.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(stokes_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def S():
    from paper_1308_4605_amd import stokes

    if not os.path.exists(stokes.LIB_PATH):
        from paper_1308_4605_amd import build

        build.build()
    return stokes


def test_library_exports_every_declared_function(S):
    names = _declared()
    assert len(names) >= 14
    lib = ctypes.CDLL(S.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(S.ABI_FUNCTIONS) == set(names)


@pytest.mark.parametrize("dim,n,bc", [(2, (32, 32), (0, 0)), (2, (1024, 1024), (1, 1)),
                                      (3, (128, 128, 128), (1, 1, 1)), (3, (256, 256, 256), (0, 0, 0)),
                                      (3, (48, 40, 8), (1, 0, 1)), (2, (2, 2), (1, 1)),
                                      (3, (48, 40, 8), (2, 0, 1)), (2, (32, 16), (2, 2)),
                                      (2, (32, 16), (0, 3)), (3, (48, 40, 8), (4, 3, 1))])
def test_sizes_match_layout(S, dim, n, bc):
    p = S.make_params(dim, n, bc, 1.0 / n[0], 0.0)
    nv, nc, ne, nl = S.stokes_sizes(p)
    lay = W.make_layout(dim, n, bc)
    assert (nv, nc, ne) == (lay.nvel, lay.ncell, lay.nedge)
    nmin = min(n)
    assert nl == int(round(__import__("math").log2(nmin)))
    assert S.stokes_workspace_bytes(p) > 8 * (lay.nvel + lay.ncell) * 12


@pytest.mark.parametrize("bad", [
    dict(dim=4), dict(n=(12, 12)), dict(n=(32, 24)), dict(h=0.0), dict(theta=-1.0),
    dict(precond=6), dict(precision=1, krylov=0), dict(restart=0), dict(restart=33),
    dict(nu_coarse=0), dict(vcycles=0), dict(edge_avg=3), dict(bc=(5, 0)), dict(bc=(-1, 0)),
    dict(n=(96, 64)), dict(dim=3, n=(1024, 1024, 1024), bc=(0, 0, 0))])
def test_invalid_parameters_rejected_on_host(S, bad):
    base = dict(dim=2, n=(32, 32), bc=(0, 0), h=1 / 32, theta=1.0)
    base.update(bad)
    p = S.make_params(**base)
    nv, nc, ne, nl = (ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int())
    rc = S.lib().stokes_sizes(ctypes.byref(p), ctypes.byref(nv), ctypes.byref(nc), ctypes.byref(ne),
                              ctypes.byref(nl))
    assert rc == S.STOKES_EINVAL
    assert S.stokes_workspace_bytes(p) == 0
    h = ctypes.c_void_p()
    rc = S.lib().stokes_create(ctypes.byref(p), None, None, None, None, None, 0, None,
                               ctypes.byref(h))
    assert rc == S.STOKES_EINVAL and not h.value


def test_strerror(S):
    assert S.strerror(0) == "ok"
    assert "max_iter" in S.strerror(S.STOKES_ENOCONV)
