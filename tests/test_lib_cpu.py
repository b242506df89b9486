"""CPU-side checks of the C ABI: the library loads, exports every function
include/pr.h declares, and rejects bad arguments before touching a device.
"""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pr.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(pr_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2510_07672_amd import _lib
    return _lib


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("pr_fine_propagate", "pr_coarse_apply", "pr_correct", "pr_solve"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(L.EXPORTED) == set(declared_functions())
    assert lib.pr_abi_version() == 13


def test_library_exports_match_nm(L):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB], capture_output=True, text=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in syms, name


def _prob(L, **kw):
    d = dict(dim=2, n=64, length=1.0, eps=0.02, conservative=0, stab=2.0, dt=1e-4, steps=10,
             fine_prec=L.PR_F64)
    d.update(kw)
    return L.Problem(**d)


@pytest.mark.parametrize("kw,status", [
    (dict(n=60), 2), (dict(n=8), 2), (dict(n=2048), 2), (dict(dim=3), 2),
    (dict(eps=0.0), 1), (dict(dt=-1.0), 1), (dict(steps=0), 1), (dict(length=float("nan")), 1),
    (dict(conservative=2), 1), (dict(stab=-1.0), 1), (dict(fine_prec=2), 2),
    (dict(scheme=2), 1), (dict(scheme=1, picard_iters=0), 1), (dict(scheme=1, picard_iters=65), 1),
    (dict(laplacian=2), 1),
])
def test_problem_validation(L, kw, status):
    lib = L.lib()
    p = _prob(L, **kw)
    st = lib.pr_fine_propagate(C.byref(p), 1, C.c_void_p(16), C.c_void_p(32), 0, C.c_void_p(64),
                               1 << 30, None)
    assert st == status
    assert lib.pr_last_error()
    assert lib.pr_fine_workspace_bytes(C.byref(p), 1) == 0


def test_null_and_alias_rejected(L):
    lib = L.lib()
    p = _prob(L)
    assert lib.pr_fine_propagate(C.byref(p), 1, None, C.c_void_p(32), 0, C.c_void_p(64), 1 << 30,
                                 None) == L.PR_ERR_INVALID_ARG
    assert lib.pr_fine_propagate(C.byref(p), 1, C.c_void_p(32), C.c_void_p(32), 0, C.c_void_p(64),
                                 1 << 30, None) == L.PR_ERR_INVALID_ARG
    assert lib.pr_fine_propagate(C.byref(p), 1, C.c_void_p(16), C.c_void_p(32), 0, None, 0,
                                 None) == L.PR_ERR_WORKSPACE
    assert lib.pr_fine_propagate(C.byref(p), -1, None, None, 0, None, 0, None) == L.PR_ERR_INVALID_ARG
    # nothing to do: success without any device call
    assert lib.pr_fine_propagate(C.byref(p), 0, None, None, 0, None, 0, None) == L.PR_OK


def test_correct_rejects_aliases(L):
    lib = L.lib()
    a, b, c = C.c_void_p(64), C.c_void_p(128), C.c_void_p(256)
    st = lib.pr_correct(1, 16, a, 0, b, b, c, C.c_void_p(512), 1, None)
    assert st == L.PR_ERR_INVALID_ARG
    assert lib.pr_correct(1, 16, a, 5, b, c, C.c_void_p(8), C.c_void_p(512), 1, None) == L.PR_ERR_INVALID_ARG


def test_solve_validation(L):
    lib = L.lib()
    p = _prob(L)
    g = L.Coarse(kind=L.PR_G_SCHEME, dt=1e-2, steps=1, prec=L.PR_F64)
    bad_g = L.Coarse(kind=7, dt=1e-2, steps=1, prec=L.PR_F64)
    args = (2, 8, C.c_void_p(16), C.c_void_p(32), 1e-10, 8, None, C.c_void_p(64), 1 << 40, None)
    assert lib.pr_solve(C.byref(p), C.byref(bad_g), *args) == L.PR_ERR_UNSUPPORTED
    assert lib.pr_solve(C.byref(p), C.byref(g), 2, 0, *args[2:]) == L.PR_ERR_INVALID_ARG
    assert lib.pr_solve(C.byref(p), C.byref(g), 2, 8, C.c_void_p(16), C.c_void_p(32), -1.0, 8,
                        None, C.c_void_p(64), 1 << 40, None) == L.PR_ERR_INVALID_ARG
    assert lib.pr_solve(C.byref(p), C.byref(g), 2, 8, C.c_void_p(16), C.c_void_p(1 << 30), 1e-10, 8,
                        None, C.c_void_p(64), 10, None) == L.PR_ERR_WORKSPACE
    # U overlapping u0
    assert lib.pr_solve(C.byref(p), C.byref(g), 2, 8, C.c_void_p(16), C.c_void_p(32), 1e-10, 8,
                        None, C.c_void_p(64), 1 << 40, None) == L.PR_ERR_INVALID_ARG
    need = lib.pr_solve_workspace_bytes(C.byref(p), C.byref(g), 2, 8)
    # U, G cache and F buffers dominate: 3 * B * s * N^2 * 8 bytes at least
    assert need >= 3 * 2 * 8 * 64 * 64 * 8


def test_status_strings(L):
    lib = L.lib()
    for s in range(7):
        assert lib.pr_status_string(s).startswith(b"PR_")


@pytest.mark.parametrize("kw,status", [
    (dict(channels=24), 2), (dict(channels=8, n_layers=3), 2), (dict(prec=0, channels=48), 2),
    (dict(prec=3, channels=64), 2), (dict(n_layers=1), 1), (dict(act=5), 1),
    (dict(limiter=1, lim_lo=1.0, lim_hi=0.0), 1), (dict(weights=None), 1),
])
def test_cnn_coarse_validation(L, kw, status):
    lib = L.lib()
    p = _prob(L)
    d = dict(kind=L.PR_G_CNN, prec=L.PR_BF16, n_layers=4, channels=32, weights=64, biases=128,
             act=L.PR_ACT_GELU, residual=1)
    d.update(kw)
    g = L.Coarse(**d)
    st = lib.pr_coarse_apply(C.byref(p), C.byref(g), 1, C.c_void_p(16), C.c_void_p(32),
                             C.c_void_p(64), 1 << 40, None)
    assert st == status, lib.pr_last_error()
    p16 = _prob(L, n=16)
    g_ok = L.Coarse(**dict(d, **{k: v for k, v in dict(channels=32, n_layers=4, prec=L.PR_BF16, act=0, limiter=0, weights=64).items()}))
    assert lib.pr_coarse_apply(C.byref(p16), C.byref(g_ok), 1, C.c_void_p(16), C.c_void_p(32),
                               C.c_void_p(64), 1 << 40, None) == L.PR_ERR_UNSUPPORTED


def _job(L, u0, U, n=64, slices=8, **pkw):
    p = _prob(L, n=n, **pkw)
    g = L.Coarse(kind=L.PR_G_SCHEME, dt=1e-2, steps=1, prec=L.PR_F64)
    return L.Job(problem=p, coarse=g, n_ics=2, n_slices=slices, max_iter=slices, tol=1e-10,
                 u0=u0, U=U, stats=None, status=-1)


def test_solve_many_validation(L):
    lib = L.lib()
    G = 1 << 30
    jobs = (L.Job * 2)(_job(L, 16 * G, 17 * G), _job(L, 18 * G, 19 * G, n=128))
    need = lib.pr_solve_many_workspace_bytes(2, jobs)
    one = lib.pr_solve_many_workspace_bytes(1, jobs)
    assert need > one > 0
    assert lib.pr_solve_many(2, jobs, C.c_void_p(20 * G), need - 1, None) == L.PR_ERR_WORKSPACE
    assert lib.pr_solve_many(0, None, None, 0, None) == L.PR_OK
    assert lib.pr_solve_many(-1, jobs, None, 0, None) == L.PR_ERR_INVALID_ARG
    # overlapping U of two jobs
    bad = (L.Job * 2)(_job(L, 16 * G, 17 * G), _job(L, 18 * G, 17 * G + 4096))
    assert lib.pr_solve_many(2, bad, C.c_void_p(20 * G), need, None) == L.PR_ERR_INVALID_ARG
    assert b"overlap" in lib.pr_last_error()
    # misaligned, schedule needs FP64 and fewer iterations than slices
    for j in (_job(L, 16 * G + 4, 17 * G), _job(L, 16 * G, 17 * G, fine_prec=L.PR_F32, f32_iters=1),
              _job(L, 16 * G, 17 * G, f32_iters=8), _job(L, 16 * G, 17 * G, f32_iters=-1)):
        arr = (L.Job * 1)(j)
        assert lib.pr_solve_many(1, arr, C.c_void_p(20 * G), 1 << 40, None) == L.PR_ERR_INVALID_ARG
    # a schedule needs no more workspace than FP64 fine solves
    arr = (L.Job * 1)(_job(L, 16 * G, 17 * G, f32_iters=3))
    assert lib.pr_solve_many_workspace_bytes(1, arr) > 0


def test_overlap_setting(L):
    lib = L.lib()
    old = lib.pr_get_overlap()
    assert lib.pr_set_overlap(0) == L.PR_ERR_INVALID_ARG
    assert lib.pr_set_overlap(17) == L.PR_ERR_INVALID_ARG
    assert lib.pr_set_overlap(3) == L.PR_OK and lib.pr_get_overlap() == 3
    assert lib.pr_set_overlap(old) == L.PR_OK


def test_coarse_plan_setting(L):
    """The network plans are AUTO, LAYERED, FUSED and FOLDED; anything else
    is rejected and leaves the setting alone."""
    lib = L.lib()
    assert (L.PR_CNN_PLAN_AUTO, L.PR_CNN_PLAN_LAYERED, L.PR_CNN_PLAN_FUSED,
            L.PR_CNN_PLAN_FOLDED) == (0, 1, 2, 3)
    for bad in (-1, 4, 99):
        assert lib.pr_set_coarse_plan(bad) == L.PR_ERR_INVALID_ARG
    for ok in (3, 2, 1, 0):
        assert lib.pr_set_coarse_plan(ok) == L.PR_OK


def test_coarse_tile_setting(L):
    """The hidden-layer tiles are AUTO, 8X32 and 16X16; anything else is
    rejected and leaves the setting alone.  The getter reports the tile a
    bf16 network's hidden layers take: 16 x 16 only where it is built (32 and
    48 channels), 0 without bf16 hidden layers, -1 for an invalid network."""
    lib = L.lib()
    assert (L.PR_CNN_TILE_AUTO, L.PR_CNN_TILE_8X32, L.PR_CNN_TILE_16X16) == (0, 1, 2)
    for bad in (-1, 3, 99):
        assert lib.pr_set_coarse_tile(bad) == L.PR_ERR_INVALID_ARG
    d = dict(kind=L.PR_G_CNN, prec=L.PR_BF16X2, n_layers=6, channels=48, weights=64, biases=128,
             act=L.PR_ACT_GELU, residual=1)
    g48, g32 = L.Coarse(**d), L.Coarse(**dict(d, channels=32, n_layers=4))
    g64, g16 = L.Coarse(**dict(d, channels=64, prec=L.PR_BF16)), L.Coarse(**dict(d, channels=16))
    g2 = L.Coarse(**dict(d, n_layers=2))
    gf = L.Coarse(**dict(d, prec=L.PR_F32))
    try:
        # untuned: 16 x 16 at 48 channels, 8 x 32 at 32
        assert lib.pr_get_coarse_tile(C.byref(g48), 512) == L.PR_CNN_TILE_16X16
        assert lib.pr_get_coarse_tile(C.byref(g32), 512) == L.PR_CNN_TILE_8X32
        assert lib.pr_set_coarse_tile(L.PR_CNN_TILE_16X16) == L.PR_OK
        assert lib.pr_set_coarse_tile(3) == L.PR_ERR_INVALID_ARG
        for g in (g48, g32):
            assert lib.pr_get_coarse_tile(C.byref(g), 512) == L.PR_CNN_TILE_16X16
            assert lib.pr_get_coarse_tile(C.byref(g), 32) == L.PR_CNN_TILE_16X16
        for g in (g64, g16):
            assert lib.pr_get_coarse_tile(C.byref(g), 512) == L.PR_CNN_TILE_8X32
        assert lib.pr_get_coarse_tile(C.byref(g2), 512) == 0
        assert lib.pr_get_coarse_tile(C.byref(gf), 512) == 0
        assert lib.pr_get_coarse_tile(C.byref(g48), 16) == -1    # the network needs N >= 32
        assert lib.pr_get_coarse_tile(C.byref(g48), 100) == -1
        assert lib.pr_set_coarse_tile(L.PR_CNN_TILE_8X32) == L.PR_OK
        assert lib.pr_get_coarse_tile(C.byref(g32), 256) == L.PR_CNN_TILE_8X32
    finally:
        assert lib.pr_set_coarse_tile(L.PR_CNN_TILE_AUTO) == L.PR_OK


def test_fft_split_setting(L):
    """The radix splits are AUTO, R8 and R4_TAIL per (N, precision); only
    N = 16, 128 and 1024 have a second split, other N report R8 whatever
    is set; bad N, precision or split values are rejected."""
    lib = L.lib()
    assert (L.PR_FFT_SPLIT_AUTO, L.PR_FFT_SPLIT_R8, L.PR_FFT_SPLIT_R4_TAIL) == (0, 1, 2)
    try:
        for n in (16, 32, 64, 128, 256, 512, 1024):
            for prec in (L.PR_F64, L.PR_F32):
                assert lib.pr_get_fft_split(n, prec) == L.PR_FFT_SPLIT_R8   # untuned
                assert lib.pr_set_fft_split(n, prec, L.PR_FFT_SPLIT_R4_TAIL) == L.PR_OK
                want = L.PR_FFT_SPLIT_R4_TAIL if n in (16, 128, 1024) else L.PR_FFT_SPLIT_R8
                assert lib.pr_get_fft_split(n, prec) == want
        assert lib.pr_set_fft_split(1000, L.PR_F64, 1) == L.PR_ERR_UNSUPPORTED
        assert lib.pr_set_fft_split(2048, L.PR_F64, 1) == L.PR_ERR_UNSUPPORTED
        assert lib.pr_set_fft_split(128, L.PR_BF16, 1) == L.PR_ERR_INVALID_ARG
        for bad in (-1, 3):
            assert lib.pr_set_fft_split(128, L.PR_F64, bad) == L.PR_ERR_INVALID_ARG
        assert lib.pr_get_fft_split(128, L.PR_F64) == L.PR_FFT_SPLIT_R4_TAIL   # unchanged
        assert lib.pr_get_fft_split(100, L.PR_F64) == -1
        assert lib.pr_get_fft_split(128, L.PR_BF16) == -1
    finally:
        for n in (16, 32, 64, 128, 256, 512, 1024):
            for prec in (L.PR_F64, L.PR_F32):
                assert lib.pr_set_fft_split(n, prec, L.PR_FFT_SPLIT_AUTO) == L.PR_OK


def test_working_set_setting(L):
    import ctypes as C
    lib = L.lib()
    assert lib.pr_get_fine_working_set(512, L.PR_F64) == 256 << 20
    assert lib.pr_get_fine_working_set(500, L.PR_F64) == -1
    assert lib.pr_set_fine_working_set(-1) == L.PR_ERR_INVALID_ARG
    assert lib.pr_set_fine_working_set(0) == L.PR_OK
    assert lib.pr_get_fine_working_set(256, L.PR_F32) == 0
    assert lib.pr_set_fine_working_set(256 << 20) == L.PR_OK


def test_bench_refuses_several_gpus():
    """The benchmark runs on one GPU: asked for more it exits with status 2
    and says so, before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_scheme_loss_validation(L):
    """pr_scheme_loss checks its arguments before any launch."""
    lib = L.lib()
    p = _prob(L)
    big = 1 << 30
    n2b = 16 * 16 * 8
    u0, u1, loss, grad = (C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20),
                          C.c_void_p(4 << 20))
    ws = C.c_void_p(8 << 20)
    need = lib.pr_scheme_loss_workspace_bytes(C.byref(p), 2)
    assert need > 2 * n2b
    f = lib.pr_scheme_loss
    assert f(C.byref(_prob(L, laplacian=1)), 1e-3, 2, u0, u1, loss, grad, None, ws, big,
             None) == L.PR_ERR_UNSUPPORTED
    assert f(C.byref(p), 0.0, 2, u0, u1, loss, grad, None, ws, big, None) == L.PR_ERR_INVALID_ARG
    assert f(C.byref(p), 1e-3, 0, u0, u1, loss, grad, None, ws, big, None) == L.PR_ERR_INVALID_ARG
    assert f(C.byref(p), 1e-3, 2, None, u1, loss, grad, None, ws, big, None) == L.PR_ERR_INVALID_ARG
    assert f(C.byref(p), 1e-3, 2, u0, u1, None, grad, None, ws, big, None) == L.PR_ERR_INVALID_ARG
    # an output inside an input, or two outputs on one another
    assert f(C.byref(p), 1e-3, 2, u0, u1, C.c_void_p((1 << 20) + 8), grad, None, ws, big,
             None) == L.PR_ERR_INVALID_ARG
    assert f(C.byref(p), 1e-3, 2, u0, u1, loss, grad, grad, ws, big, None) == L.PR_ERR_INVALID_ARG
    assert f(C.byref(p), 1e-3, 2, u0, u1, loss, grad, None, ws, need - 1,
             None) == L.PR_ERR_WORKSPACE
    assert lib.pr_last_error()


def test_fine_queue_setting(L):
    lib = L.lib()
    assert lib.pr_get_fine_queue() == 0
    assert lib.pr_set_fine_queue(3) == L.PR_ERR_INVALID_ARG
    assert lib.pr_set_fine_queue(-1) == L.PR_ERR_INVALID_ARG
    assert lib.pr_get_fine_queue() == 0
    # off and nothing tuned: pass by pass for every class
    assert lib.pr_get_fine_queue_choice(512, L.PR_F64) == 0
    assert lib.pr_get_fine_queue_choice(500, L.PR_F64) == -1
    assert lib.pr_get_fine_queue_choice(512, L.PR_BF16) == -1
    assert lib.pr_set_fine_queue(2) == L.PR_OK and lib.pr_get_fine_queue() == 2
    assert lib.pr_get_fine_queue_choice(256, L.PR_F64) == 1
    assert lib.pr_set_fine_queue(1) == L.PR_OK and lib.pr_get_fine_queue() == 1
    assert lib.pr_get_fine_queue_choice(512, L.PR_F64) == 1
    assert lib.pr_get_fine_queue_choice(32, L.PR_F64) == 0      # outside the queue's sizes
    assert lib.pr_get_fine_queue_choice(512, L.PR_F32) == 0     # FP32 at 512^2: 512-thread tiles
    assert lib.pr_set_fine_queue(0) == L.PR_OK and lib.pr_get_fine_queue() == 0
