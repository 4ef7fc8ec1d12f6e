"""The C-ABI library loads and exports every entry point include/gmhc.h declares, and
its host-only validation behaves as documented (no GPU compute is called here)."""
import ctypes as C
import os
import re

import pytest

from paper_2609_36383_amd import gmhc as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "gmhc.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(gmhc_[a-z_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    assert _declared() == sorted(G.SYMBOLS)


def test_library_exports_every_symbol():
    lib = G.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.gmhc_abi_version() == G.ABI_VERSION


def test_host_validation():
    lib = G.load_library()
    h = C.c_void_p()
    good = G.make_config(2, (16, 16), (0, 0), (3.2, 3.2), 0.05)
    assert lib.gmhc_create(C.byref(good), C.byref(h)) == G.OK
    n = C.c_size_t()
    assert lib.gmhc_workspace_bytes(h, 1000, C.byref(n)) == G.OK and n.value > 0
    n2 = C.c_size_t()
    assert lib.gmhc_workspace_bytes(h, 100000, C.byref(n2)) == G.OK and n2.value > n.value
    lib.gmhc_destroy(h)
    for sh in (0, 1, 2):  # 0 selects the quadratic shape
        c = G.make_config(2, (16, 16), (0, 0), (3.2, 3.2), 0.05, shape_order=sh)
        hh = C.c_void_p()
        assert lib.gmhc_create(C.byref(c), C.byref(hh)) == G.OK, sh
        lib.gmhc_destroy(hh)
    # shape_order and deterministic took the places of two reserved ints: the struct
    # layout is unchanged
    assert G.Config.shape_order.offset == G.Config.ls_halvings.offset + 4
    assert G.Config.anderson_lambda.offset == G.Config.deterministic.offset + 4
    for det in (0, 1):
        c = G.make_config(2, (16, 16), (0, 0), (3.2, 3.2), 0.05, deterministic=det)
        hh = C.c_void_p()
        assert lib.gmhc_create(C.byref(c), C.byref(hh)) == G.OK, det
        lib.gmhc_destroy(hh)
    # refine_levels closes the structure (the compiler pads it to a multiple of 8)
    assert G.Config.refine_levels.offset == G.Config.ls_growth.offset + 8
    assert C.sizeof(G.Config) == G.Config.refine_levels.offset + 8
    for rl in range(4):
        c = G.make_config(2, (16, 16), (0, 0), (3.2, 3.2), 0.05, refine_levels=rl)
        hh = C.c_void_p()
        assert lib.gmhc_create(C.byref(c), C.byref(hh)) == G.OK, rl
        n1, n2 = C.c_size_t(), C.c_size_t()
        assert lib.gmhc_workspace_bytes(hh, 1000, C.byref(n1)) == G.OK
        lib.gmhc_destroy(hh)
        if rl:  # the refinement buffers are only taken when it is on
            assert n1.value > n0.value
        else:
            n0 = n1
    bad = [
        dict(sigma1=2.0),                 # sigma1 != kappa^2 sigma2
        dict(dt=0.0),
        dict(n=(12, 16)),                 # not a power of two
        dict(gl_order=9),
        dict(beta=0.0),
        dict(max_outer=0),
        dict(outer_scheme=2),
        dict(outer_scheme=1, anderson_m=0),
        dict(outer_scheme=1, anderson_m=9),
        dict(outer_scheme=1, ls_growth=0.9),
        dict(outer_scheme=1, ls_decrease=1.0),
        dict(timing=-1),
        dict(shape_order=3),
        dict(shape_order=-1),
        dict(deterministic=2),
        dict(refine_levels=-1),
        dict(refine_levels=4),
    ]
    for over in bad:
        kw = dict(dim=2, n=(16, 16), lo=(0, 0), length=(3.2, 3.2), dt=0.05)
        kw.update(over)
        c = G.make_config(**kw)
        hh = C.c_void_p()
        assert lib.gmhc_create(C.byref(c), C.byref(hh)) == G.EINVAL, over
    # more than 2^30 mesh nodes (node indices are int32 in the kernels)
    c = G.make_config(3, (4096, 4096, 128), (0, 0, 0), (1, 1, 1), 0.1)
    hh = C.c_void_p()
    assert lib.gmhc_create(C.byref(c), C.byref(hh)) == G.EINVAL
    c = G.make_config(4, (16, 16, 16), (0, 0, 0), (1, 1, 1), 0.1)
    c.dim = 4
    assert lib.gmhc_create(C.byref(c), C.byref(C.c_void_p())) == G.EINVAL


def test_calls_out_of_order_are_rejected():
    lib = G.load_library()
    h = C.c_void_p()
    c = G.make_config(1, (16,), (0,), (1.0,), 0.1)
    assert lib.gmhc_create(C.byref(c), C.byref(h)) == G.OK
    assert lib.gmhc_initialize(h) == G.ESTATE
    assert lib.gmhc_step(h, None) == G.ESTATE
    n = C.c_size_t()
    assert lib.gmhc_state_bytes(h, C.byref(n)) == G.ESTATE  # not bound
    buf = (C.c_uint8 * 64)()
    assert lib.gmhc_save(h, buf, 64, G.HOST) == G.ESTATE
    assert lib.gmhc_load(h, buf, 64, G.HOST) == G.ESTATE
    assert b"initialize" in lib.gmhc_last_error(h) or lib.gmhc_last_error(h)
    # the adjoint calls need an initialized (or loaded) state
    dummy = (C.c_double * 8)()
    assert lib.gmhc_energy_grad(h, dummy, G.HOST) == G.ESTATE
    assert lib.gmhc_adjoint_step(h, buf, 64, *([dummy] * 9), None) == G.ESTATE
    assert lib.gmhc_adjoint_initialize(h, buf, 64, *([dummy] * 6)) == G.ESTATE
    assert lib.gmhc_adjoint_step(h, buf, 64, *([dummy] * 8), None, None) == G.EINVAL  # null output
    n = C.c_size_t()
    assert lib.gmhc_adjoint_bytes(h, C.byref(n)) == G.OK and n.value > 0
    lib.gmhc_destroy(h)
