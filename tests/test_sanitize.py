"""Memory safety and defined behaviour of the CPU-side code under
AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle (oracle/ibo.c, plain C) is built with gcc and both sanitizers
  (recovery off, leak detection on) together with tests/sanitize_oracle.c,
  which calls every oracle entry point on small ragged problems (2-D and
  3-D, periodic and channel walls, tethers, Stokes mode, every line-solve
  boundary kind); the run must exit cleanly.
* The library's host code (argument validation, the line-solve factor
  tables, the structure upload's CSR build up to its first device call) is
  built with the sanitizers on the host side only (`-Xarch_host`; the gfx950
  device code is built as usual) and driven through the C ABI in a child
  process that preloads the sanitizer runtime: every call here is refused on
  the host before it reaches the device, so no GPU is needed.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_1305_3976_amd", "_build", "sanitize")


def test_oracle_under_address_and_undefined_sanitizers():
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "sanitize_oracle")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", "-Wall", "-I", os.path.join(ROOT, "oracle"),
           "-o", exe, os.path.join(ROOT, "tests", "sanitize_oracle.c"),
           os.path.join(ROOT, "oracle", "ibo.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert r.stdout.startswith("checksum ")


HOST_CHECKS = textwrap.dedent(r'''
    import ctypes, sys
    sys.path.insert(0, sys.argv[2])
    L = ctypes.CDLL(sys.argv[1])
    from paper_1305_3976_amd import ibgm      # structures only (loads the normal build too)
    ok = 0
    def expect(st, want):
        global ok
        assert st == want, (st, want, L.ib_last_error())
        ok += 1
    L.ib_last_error.restype = ctypes.c_char_p
    n = ctypes.c_size_t()
    # parameter validation, every field
    for field, val in [("dim", 1), ("h", 0.0), ("rho", -1.0), ("dt", float("nan")),
                       ("mu", -0.1), ("chi", 1.5), ("precision", 7), ("flags", 0x100),
                       ("step0", -1)]:
        Q = ibgm.Config(2, (64, 64), 1 / 64).params()
        setattr(Q, field, val)
        expect(L.ib_workspace_size(ctypes.byref(Q), ctypes.c_int64(10), ctypes.byref(n)), 1)
    for dims in [(3, (256, 256, 256)), (2, (48, 40, 7)), (3, (24, 20, 28))]:
        for prec in (0, 1, 2):
            P = ibgm.Config(dims[0], dims[1], 1 / dims[1][0], mu=0.01, dt=1e-3,
                            precision=prec).params()
            expect(L.ib_workspace_size(ctypes.byref(P), ctypes.c_int64(65536), ctypes.byref(n)), 0)
    # ib_init: null buffers, bad structures (refused before any device call)
    P = ibgm.Config(2, (16, 16), 1 / 16).params()
    B = ibgm.Buffers()
    S = ibgm.Structure()
    ctx = ctypes.c_void_p()
    expect(L.ib_init(ctypes.byref(ctx), ctypes.byref(P), ctypes.byref(B), ctypes.byref(S), None), 1)
    # line solve: every refusal
    nn = (ctypes.c_int32 * 3)(8, 8, 1)
    fake = ctypes.c_void_p(0x1000)
    for args in [(fake, 0, nn, 0, 1, 64, 1.0, -0.6), (fake, 5, nn, 0, 1, 64, 3.0, -1.0),
                 (fake, 0, nn, 3, 1, 64, 3.0, -1.0), (fake, 0, nn, 2, 1, 64, 3.0, -1.0),
                 (fake, 0, nn, 0, 2, 10, 3.0, -1.0), (None, 0, nn, 0, 1, 64, 3.0, -1.0)]:
        a = list(args)
        expect(L.ib_line_solve(a[0], ctypes.c_int32(a[1]), a[2], ctypes.c_int32(a[3]),
                               ctypes.c_int32(a[4]), ctypes.c_int64(a[5]), ctypes.c_double(a[6]),
                               ctypes.c_double(a[7]), None), 1)
    # allocation-free spreading: beyond the static array, batches, null pointers
    ptrs = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    P3 = ibgm.Config(3, (256, 256, 256), 1 / 256, mu=0.01, dt=5e-4).params()
    expect(L.ib_spread_static(ctypes.byref(P3), fake, fake, fake,
                              ctypes.c_int64(ibgm.IB_SPREAD_STATIC_MAX_BYTES + 1), ptrs,
                              0, None), 2)
    Q = ibgm.Config(2, (64, 64, 3), 1 / 64, mu=0.01, dt=1e-3).params()
    expect(L.ib_spread_static(ctypes.byref(Q), fake, fake, fake, ctypes.c_int64(10), ptrs, 0,
                              None), 1)
    # null contexts
    expect(L.ib_step(None, ctypes.c_int32(1)), 5)
    expect(L.ib_restart(None, ctypes.c_int64(1)), 5)
    expect(L.ib_refresh_divergence(None), 5)
    expect(L.ib_sync(None, None), 5)
    print("host checks", ok)
''')


def test_host_code_under_address_and_undefined_sanitizers():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    clang = "/opt/rocm/llvm/bin/clang"
    rt = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    if not os.path.exists(rt):
        pytest.skip("clang AddressSanitizer runtime not found")
    os.makedirs(BUILD, exist_ok=True)
    lib = os.path.join(BUILD, "libibgm_san.so")
    csrc = os.path.join(ROOT, "paper_1305_3976_amd", "csrc")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan",
           "-I", os.path.join(ROOT, "include"), "-I", csrc, "-o", lib,
           os.path.join(csrc, "ibgm.hip"), os.path.join(csrc, "closure.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", HOST_CHECKS, lib, ROOT], capture_output=True,
                       text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "host checks" in r.stdout
