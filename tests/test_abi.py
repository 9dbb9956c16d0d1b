"""The C-ABI library loads and exports every entry point include/gea.h
declares; argument errors are reported without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gea_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_2303_10499_amd import gea
    if not os.path.exists(gea.LIB_PATH):
        from paper_2303_10499_amd import build
        build.build()
    return gea.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared("gea.h")
    assert "gea_step" in names and "gea_pressure_solve" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in gea.h but not exported"


def test_workspace_bytes_and_argument_errors(L):
    from paper_2303_10499_amd import configs, gea
    cfg = configs.get("bubble2d_64x32")
    m, p = gea.make_mesh(cfg["mesh"]), gea.make_params(cfg["params"])
    n = C.c_size_t(0)
    assert L.gea_workspace_bytes(C.byref(m), C.byref(p), C.byref(n)) == gea.OK
    assert n.value > 40 * 8 * 64 * 32
    bad = gea.make_mesh(dict(cfg["mesh"], nx=0))
    assert L.gea_workspace_bytes(C.byref(bad), C.byref(p), C.byref(n)) == gea.ERR_ARG
    assert b"positive" in L.gea_last_error(None)
    p2 = gea.make_params(dict(cfg["params"], dt=-1.0))
    assert L.gea_workspace_bytes(C.byref(m), C.byref(p2), C.byref(n)) == gea.ERR_ARG
    ctx = C.c_void_p()
    # no workspace
    assert L.gea_init_mesh(C.byref(m), C.byref(p), None, None, 0, C.byref(ctx)) == gea.ERR_ARG
    assert not ctx.value
    # null context
    assert L.gea_step(None, 1, None) == gea.ERR_ARG


def test_workspace_fits_the_largest_workload(L):
    from paper_2303_10499_amd import configs, gea
    cfg = configs.get("bubble3d_384x384x192")
    m, p = gea.make_mesh(cfg["mesh"]), gea.make_params(cfg["params"], "mixed")
    n = C.c_size_t(0)
    assert L.gea_workspace_bytes(C.byref(m), C.byref(p), C.byref(n)) == gea.OK
    assert n.value < 64 * 2**30   # well inside one GPU's 288 GB
