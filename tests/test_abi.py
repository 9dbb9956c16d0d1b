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


@pytest.mark.parametrize("header,must", [
    ("gea.h", ("gea_init_mesh", "gea_set_state", "gea_step", "gea_pressure_solve",
               "gea_get_fields", "gea_time_network")),
    ("gea_learned.h", ("gea_cnn_forward", "gea_cnn_backward", "gea_cnn_adam",
                       "gea_load_weights", "gea_make_pair", "gea_learned_apply",
                       "gea_learned_activation")),
])
def test_every_declared_symbol_is_exported(L, header, must):
    names = declared(header)
    for n in must:
        assert n in names, f"{n} missing from {header}"
    for n in names:
        assert hasattr(L, n), f"{n} declared in {header} but not exported"


def test_network_argument_errors(L):
    from paper_2303_10499_amd import gea, learned
    Ll = learned._lib()
    n = C.c_int64(0)
    assert Ll.gea_cnn_param_count(2, C.byref(n)) == gea.OK and n.value == 58193
    assert Ll.gea_cnn_param_count(3, C.byref(n)) == gea.OK and n.value == 174257
    assert Ll.gea_cnn_param_count(4, C.byref(n)) == gea.ERR_ARG
    b = C.c_size_t(0)
    # grid dimensions must be multiples of 4 (two 2x poolings)
    assert Ll.gea_cnn_workspace_bytes(2, 64, 1, 32, 0, C.byref(b)) == gea.OK
    assert Ll.gea_cnn_workspace_bytes(2, 66, 1, 32, 0, C.byref(b)) == gea.ERR_ARG
    assert Ll.gea_cnn_workspace_bytes(3, 16, 6, 16, 1, C.byref(b)) == gea.ERR_ARG
    # inference instances keep no concatenated inputs: smaller than training ones
    bi, bt = C.c_size_t(0), C.c_size_t(0)
    assert Ll.gea_cnn_workspace_bytes(3, 32, 32, 32, 0, C.byref(bi)) == gea.OK
    assert Ll.gea_cnn_workspace_bytes(3, 32, 32, 32, 1, C.byref(bt)) == gea.OK
    assert bi.value < bt.value
    h = C.c_void_p()
    assert Ll.gea_cnn_create(2, 64, 1, 32, 0, None, None, 0, C.byref(h)) == gea.ERR_ARG
    assert not h.value
    assert L.gea_time_network(None, 1, None, None) == gea.ERR_ARG


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


def test_static_solve_argument_errors(L):
    """the allocation-free solve rejects bad arguments and meshes beyond its
    static work area before any device work"""
    from paper_2303_10499_amd import gea
    buf = (C.c_double * 4)()
    p = C.cast(buf, C.c_void_p)
    st = gea.SolveStats()
    big = gea.Mesh(1024, 1, 1025, 1.0, 1.0, 1.0)
    rc = L.gea_pressure_solve_static(C.byref(big), p, p, p, p, 1e-8, 100, None, C.byref(st))
    assert rc == gea.ERR_ARG and b"static work area" in L.gea_last_error(None)
    ok = gea.Mesh(64, 1, 32, 1.0, 1.0, 1.0)
    assert L.gea_pressure_solve_static(C.byref(ok), None, p, p, p, 1e-8, 100, None, C.byref(st)) == gea.ERR_ARG
    assert L.gea_pressure_solve_static(C.byref(ok), p, p, p, p, 0.0, 100, None, C.byref(st)) == gea.ERR_ARG
    neg = gea.Mesh(0, 1, 32, 1.0, 1.0, 1.0)
    assert L.gea_pressure_solve_static(C.byref(neg), p, p, p, p, 1e-8, 100, None, C.byref(st)) == gea.ERR_ARG


def test_scheme_variants_and_state_entry_points_without_a_gpu(L):
    """energy_form and transport take 0 or 1; implicit transport adds its
    BiCGStab vectors (9) and the predictors' right-hand sides (ndim) to the
    workspace; the state entry points reject a null context or pointer"""
    from paper_2303_10499_amd import configs, gea
    cfg = configs.get("bubble3d_256x256x128")
    m = gea.make_mesh(cfg["mesh"])
    n0, n1 = C.c_size_t(0), C.c_size_t(0)
    p0 = gea.make_params(dict(cfg["params"], transport=0))
    p1 = gea.make_params(dict(cfg["params"], transport=1))
    assert L.gea_workspace_bytes(C.byref(m), C.byref(p0), C.byref(n0)) == gea.OK
    assert L.gea_workspace_bytes(C.byref(m), C.byref(p1), C.byref(n1)) == gea.OK
    nc = 256 * 256 * 128
    assert n1.value - n0.value >= (9 + 3) * 8 * nc
    for bad in (dict(energy_form=2), dict(transport=-1)):
        pb = gea.make_params(dict(cfg["params"], **bad))
        assert L.gea_workspace_bytes(C.byref(m), C.byref(pb), C.byref(n0)) == gea.ERR_ARG
        assert re.search(rb"energy_form|transport", L.gea_last_error(None))
    buf = (C.c_double * 4)()
    p = C.cast(buf, C.c_void_p)
    assert L.gea_set_face_flux(None, p, gea.HOST) == gea.ERR_ARG
    assert L.gea_set_history(None, p, p, gea.HOST) == gea.ERR_ARG
    assert L.gea_state_extrema(None, None) == gea.ERR_ARG
