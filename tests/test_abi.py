"""The C-ABI library loads, exports every entry point include/*.h
declares, and rejects bad arguments on the host before touching a device
(no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for h in sorted(os.listdir(inc)):
        if h.endswith(".h"):
            src = open(os.path.join(inc, h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            src = re.sub(r"#define[^\n]*", "", src)
            names |= set(re.findall(r"\b(ib_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def ib():
    # a clean checkout has no built library yet: build it (hipcc cross-compiles
    # gfx950 code on a machine without a GPU) before the binding loads it
    from paper_1305_3976_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_1305_3976_amd import ibgm
    return ibgm


def test_every_declared_symbol_is_exported(ib):
    names = declared_functions()
    assert len(names) >= 28
    for n in names:
        assert hasattr(ib.lib, n), n
    assert set(ib.EXPORTED) == set(names)


def test_workspace_size_and_validation(ib):
    P = ib.Config(3, (256, 256, 256), 1 / 256, mu=0.01, dt=5e-4, precision=ib.IB_PREC_MIXED).params()
    n = ctypes.c_size_t()
    assert ib.lib.ib_workspace_size(ctypes.byref(P), 65536, ctypes.byref(n)) == ib.IB_OK
    assert n.value >= 7 * 256 ** 3 * 4 + 3 * 3 * 65536 * 8
    bad = [("dim", 1), ("h", 0.0), ("rho", -1.0), ("dt", float("nan")), ("mu", -0.1),
           ("chi", 1.5), ("precision", 7), ("flags", 0x100), ("step0", -1)]
    for field, val in bad:
        Q = ib.Config(2, (64, 64), 1 / 64).params()
        setattr(Q, field, val)
        assert ib.lib.ib_workspace_size(ctypes.byref(Q), 10, ctypes.byref(n)) == ib.IB_E_INVALID
        assert ib.lib.ib_last_error()
    Q = ib.Config(2, (64, 3), 1 / 64).params()
    assert ib.lib.ib_workspace_size(ctypes.byref(Q), 10, ctypes.byref(n)) == ib.IB_E_INVALID
    assert b"n[1]" in ib.lib.ib_last_error()


def test_line_solve_argument_errors(ib):
    n = (ctypes.c_int32 * 3)(8, 8, 1)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert ib.lib.ib_line_solve(fake, 0, n, 0, 1, 64, 1.0, -0.6, None) == ib.IB_E_INVALID
    assert b"|diag| > 2|off|" in ib.lib.ib_last_error()
    assert ib.lib.ib_line_solve(fake, 5, n, 0, 1, 64, 3.0, -1.0, None) == ib.IB_E_INVALID
    assert ib.lib.ib_line_solve(fake, 0, n, 3, 1, 64, 3.0, -1.0, None) == ib.IB_E_INVALID
    assert ib.lib.ib_line_solve(fake, 0, n, 2, 1, 64, 3.0, -1.0, None) == ib.IB_E_INVALID
    assert ib.lib.ib_line_solve(fake, 0, n, 0, 2, 10, 3.0, -1.0, None) == ib.IB_E_INVALID
    assert ib.lib.ib_line_solve(None, 0, n, 0, 1, 64, 3.0, -1.0, None) == ib.IB_E_INVALID


def test_init_argument_errors(ib):
    P = ib.Config(2, (16, 16), 1 / 16).params()
    B = ib.Buffers()
    S = ib.Structure()
    ctx = ctypes.c_void_p()
    assert ib.lib.ib_init(ctypes.byref(ctx), ctypes.byref(P), ctypes.byref(B), ctypes.byref(S),
                          None) == ib.IB_E_INVALID
    assert not ctx.value
    assert ib.lib.ib_step(None, 1) == ib.IB_E_STATE
    assert ib.lib.ib_sync(None, None) == ib.IB_E_STATE


def test_point_count_limit(ib):
    """More points than the 32-bit sort ranks hold is refused up front (no
    array is read: the device pointers below are never dereferenced)."""
    P = ib.Config(3, (16, 16, 16), 1 / 16).params()
    n = ctypes.c_size_t()
    big = 2 ** 31
    assert ib.lib.ib_workspace_size(ctypes.byref(P), big, ctypes.byref(n)) == ib.IB_E_UNSUPPORTED
    assert ib.lib.ib_workspace_size(ctypes.byref(P), big - 1, ctypes.byref(n)) == ib.IB_OK
    B = ib.Buffers()
    fake = ctypes.c_void_p(4096)
    for c in range(3):
        B.u[c] = fake
        B.nl_prev[c] = fake
    B.psi = B.div_prev = B.p = B.X = B.U_prev = fake
    B.n_points = big
    ctx = ctypes.c_void_p()
    st = ib.lib.ib_init(ctypes.byref(ctx), ctypes.byref(P), ctypes.byref(B),
                        ctypes.byref(ib.Structure()), None)
    assert st == ib.IB_E_UNSUPPORTED and not ctx.value
    assert b"n_points" in ib.lib.ib_last_error(None)


def test_static_array_size_matches_header():
    """The Python copy of IB_SPREAD_STATIC_MAX_BYTES is the header's value
    (tests size their refusal cases by it)."""
    import os
    import re
    from paper_1305_3976_amd import ibgm
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "include", "ibgm.h")).read()
    m = re.search(r"#define IB_SPREAD_STATIC_MAX_BYTES \((\d+)u << (\d+)\)", hdr)
    assert m
    assert ibgm.IB_SPREAD_STATIC_MAX_BYTES == int(m.group(1)) << int(m.group(2))


def test_closure_argument_errors(ib):
    """The gather and the fused last layer refuse bad arguments on the host
    (the fake device pointers below are never dereferenced)."""
    L = ib.lib
    fake = ctypes.c_void_p(4096)
    n = (ctypes.c_int32 * 3)(16, 16, 16)
    U = (ib._vp * 3)(4096, 8192, 12288)
    assert L.ib_closure_conv_apply(fake, n, fake, None, 0.5, None, None) == ib.IB_E_INVALID
    same = (ib._vp * 3)(4096, 4096, 12288)
    assert L.ib_closure_conv_apply(fake, n, fake, None, 0.5, same, None) == ib.IB_E_INVALID
    assert b"distinct" in L.ib_last_error()
    assert L.ib_closure_conv_apply(fake, n, fake, None, float("inf"), U, None) == ib.IB_E_INVALID
    assert L.ib_closure_conv_apply(None, n, fake, None, 0.5, U, None) == ib.IB_E_INVALID
    bad_n = (ctypes.c_int32 * 3)(16, 0, 16)
    assert L.ib_closure_conv_apply(fake, bad_n, fake, None, 0.5, U, None) == ib.IB_E_INVALID
    odd = ctypes.c_void_p(4100)
    assert L.ib_closure_conv_apply(odd, n, fake, None, 0.5, U, None) == ib.IB_E_INVALID
    # gather
    S = (ib._vp * 13)(*([4096] * 13))
    F = (ctypes.c_float * 13)(*([1.0] * 13))
    C = (ctypes.c_int32 * 13)(*([0] * 13))
    d = (ctypes.c_int32 * 3)(8, 8, 8)
    for nsrc, out_f32, out_ch in [(0, 1, 4), (13, 1, 4), (2, 0, 8), (2, 1, 17)]:
        assert L.ib_closure_gather(S, F, C, nsrc, n, fake, 1, d, out_f32, out_ch, fake,
                                   None) == ib.IB_E_INVALID
    C[1] = 4
    assert L.ib_closure_gather(S, F, C, 2, n, fake, 1, d, 1, 4, fake, None) == ib.IB_E_INVALID
    assert b"chan[1]" in L.ib_last_error()
    C[1] = 0
    S[1] = None
    assert L.ib_closure_gather(S, F, C, 2, n, fake, 1, d, 1, 4, fake, None) == ib.IB_E_INVALID
    S[1] = 4096
    assert L.ib_closure_gather(S, F, C, 2, n, fake, 0, d, 1, 4, fake, None) == ib.IB_E_INVALID
    assert L.ib_closure_gather(S, F, C, 2, bad_n, fake, 1, d, 1, 4, fake, None) == ib.IB_E_INVALID
    assert L.ib_closure_gather(S, F, C, 2, n, fake, 1, d, 0, 16, odd, None) == ib.IB_E_INVALID
