"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
symbol of include/sym.h, computes coefficients and workspace sizes, and rejects bad
arguments before launching anything. Pointers passed here are never dereferenced:
each call fails validation first."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L_():
    from paper_1808_02281_amd import _lib

    try:
        return _lib.lib()
    except ImportError as e:
        pytest.fail(f"libsym.so not built: {e}")


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "sym.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_]+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol(L_):
    from paper_1808_02281_amd import _lib

    declared = _declared_functions()
    assert sorted(_lib.EXPORTS) == declared
    for name in declared:
        assert hasattr(L_, name), name


def test_coeffs_match_oracle(L_):
    from paper_1808_02281_amd import api

    for u0 in (0.8677, 0.862, 1.0, 1.3):
        c, a = api.coeffs(u0)
        co, ao = oracle.coeffs(u0)
        np.testing.assert_allclose(c, co, rtol=1e-15, atol=0)
        assert abs(a - ao) <= 1e-15 * max(1, abs(ao))
    c3 = (ctypes.c_double * 3)()
    assert L_.sym_coeffs(0.0, c3, None) == -1
    assert L_.sym_coeffs(float("nan"), c3, None) == -1
    assert L_.sym_coeffs(-1.0, c3, None) == -1
    assert L_.sym_coeffs(0.9, None, None) == -2


def _dims(*v):
    return (ctypes.c_int32 * 4)(*v)


def test_workspace_bytes(L_):
    ws32 = L_.sym_workspace_bytes(_dims(4, 4, 4, 4), 1)
    ws64 = L_.sym_workspace_bytes(_dims(4, 4, 4, 4), 2)
    assert ws32 > 0 and ws64 > ws32
    # the plaquette-staple buffer dominates: 8 slots x two rows (12 reals) per link
    big = L_.sym_workspace_bytes(_dims(32, 32, 32, 64), 1)
    assert big >= 4 * 32 * 32 * 32 * 64 * 8 * 12 * 4
    for bad in [(3, 4, 4, 4), (4, 4, 4, 2), (4, 5, 4, 4), (0, 4, 4, 4)]:
        assert L_.sym_workspace_bytes(_dims(*bad), 1) == 0
    assert L_.sym_workspace_bytes(_dims(4, 4, 4, 4), 3) == 0
    assert L_.sym_workspace_bytes(None, 1) == 0
    # V/2 is limited to 2^24 sites per parity: 64^3 x 128 is the largest 4D lattice of
    # that volume, one step beyond it is rejected
    assert L_.sym_workspace_bytes(_dims(64, 64, 64, 128), 1) > 0
    assert L_.sym_workspace_bytes(_dims(64, 64, 64, 130), 1) == 0


# Aligned device-looking addresses, never dereferenced: every call below fails
# validation first. They are 16 MiB apart, more than any 4^4 field or workspace, so that
# only the calls meant to test overlapping regions trip the overlap check.
FAKE = ctypes.c_void_p(0x10000000)
FAKE2 = ctypes.c_void_p(0x11000000)
FAKE3 = ctypes.c_void_p(0x12000000)
FAKE4 = ctypes.c_void_p(0x13000000)
MISALIGNED = ctypes.c_void_p(0x10000008)
HUGE = 1 << 60


def test_force_validation(L_):
    ok = _dims(4, 4, 4, 4)
    f = L_.sym_force
    assert f(_dims(4, 4, 3, 4), 0.8677, 3.0, 1, FAKE, FAKE2, None, FAKE3, HUGE, None) == -1
    assert f(None, 0.8677, 3.0, 1, FAKE, FAKE2, None, FAKE3, HUGE, None) == -2
    assert f(ok, 0.8677, 3.0, 7, FAKE, FAKE2, None, FAKE3, HUGE, None) == -1
    assert f(ok, -0.5, 3.0, 1, FAKE, FAKE2, None, FAKE3, HUGE, None) == -1
    assert f(ok, 0.8677, math.inf, 1, FAKE, FAKE2, None, FAKE3, HUGE, None) == -1
    assert f(ok, 0.8677, 3.0, 1, None, FAKE2, None, FAKE3, HUGE, None) == -2
    assert f(ok, 0.8677, 3.0, 1, FAKE, None, None, FAKE3, HUGE, None) == -2
    assert f(ok, 0.8677, 3.0, 1, MISALIGNED, FAKE2, None, FAKE3, HUGE, None) == -1
    assert f(ok, 0.8677, 3.0, 1, FAKE, FAKE2, MISALIGNED, FAKE3, HUGE, None) == -1
    assert f(ok, 0.8677, 3.0, 1, FAKE, FAKE2, None, None, HUGE, None) == -2
    assert f(ok, 0.8677, 3.0, 1, FAKE, FAKE2, None, FAKE3, 16, None) == -3


def _at(base, off):
    return ctypes.c_void_p(base.value + off)


@pytest.mark.parametrize("fn", ["sym_force", "sym_action_grad"])
def test_force_rejects_overlapping_regions(L_, fn):
    """The force kernels read neighbouring links while they write: the output may not
    alias or overlap the links, the scalars or the workspace."""
    ok = _dims(4, 4, 4, 4)
    f = getattr(L_, fn)
    field = 4 * 4 * 4 * 4 * 4 * 18 * 4  # FP32 4^4 link field, bytes
    assert f(ok, 0.8677, 3.0, 1, FAKE, FAKE, None, FAKE3, HUGE, None) == -1          # out == U
    assert f(ok, 0.8677, 3.0, 1, FAKE, _at(FAKE, field - 16), None, FAKE3, HUGE, None) == -1
    assert f(ok, 0.8677, 3.0, 1, FAKE, FAKE2, _at(FAKE2, 64), FAKE3, HUGE, None) == -1  # S inside out
    assert f(ok, 0.8677, 3.0, 1, FAKE, FAKE2, None, _at(FAKE2, 256), HUGE, None) == -1  # ws inside out
    assert f(ok, 0.8677, 3.0, 1, _at(FAKE3, 4096), FAKE2, None, FAKE3, HUGE, None) == -1  # U inside ws


def test_action_and_leapfrog_validation(L_):
    ok = _dims(4, 4, 4, 4)
    a = L_.sym_action
    assert a(ok, 0.8677, 3.0, 2, FAKE, None, FAKE3, HUGE, None) == -2  # S_dev is required
    assert a(ok, 0.8677, 3.0, 2, FAKE, FAKE2, FAKE3, 8, None) == -3
    assert a(_dims(4, 4, 4, 6), 0.0, 3.0, 2, FAKE, FAKE2, FAKE3, HUGE, None) == -1
    assert a(ok, 0.8677, 3.0, 2, FAKE, _at(FAKE3, 64), FAKE3, HUGE, None) == -1  # S inside ws
    m = L_.md_leapfrog
    assert m(ok, 0.8677, 3.0, 2, FAKE, FAKE2, math.nan, 3, None, FAKE3, HUGE, None) == -1
    assert m(ok, 0.8677, 3.0, 2, FAKE, FAKE2, 0.01, -1, None, FAKE3, HUGE, None) == -1
    assert m(ok, 0.8677, 3.0, 2, FAKE, None, 0.01, 3, None, FAKE3, HUGE, None) == -2
    assert m(ok, 0.8677, 3.0, 2, FAKE, FAKE2, 0.01, 3, None, FAKE3, 0, None) == -3
    assert m(ok, 0.8677, 3.0, 2, FAKE, FAKE, 0.01, 3, None, FAKE3, HUGE, None) == -1   # P == U
    assert m(ok, 0.8677, 3.0, 2, FAKE, _at(FAKE, 1024), 0.01, 3, None, FAKE3, HUGE, None) == -1
    assert m(ok, 0.8677, 3.0, 2, FAKE, FAKE2, 0.01, 3, _at(FAKE, 16), FAKE3, HUGE, None) == -1  # H inside U


def test_check_links_validation(L_):
    ok = _dims(4, 4, 4, 4)
    c = L_.sym_check_links
    assert c(_dims(4, 4, 4, 5), 1, FAKE, FAKE2, FAKE3, HUGE, None) == -1
    assert c(ok, 3, FAKE, FAKE2, FAKE3, HUGE, None) == -1
    assert c(ok, 1, None, FAKE2, FAKE3, HUGE, None) == -2
    assert c(ok, 1, FAKE, None, FAKE3, HUGE, None) == -2
    assert c(ok, 1, FAKE, FAKE2, FAKE3, 8, None) == -3
    assert c(ok, 1, FAKE, _at(FAKE, 32), FAKE3, HUGE, None) == -1


def test_reunitarise_validation(L_):
    ok = _dims(4, 4, 4, 4)
    r = L_.sym_reunitarise
    assert r(_dims(4, 4, 4, 5), 1, FAKE, None) == -1
    assert r(_dims(4, 4, 2, 4), 2, FAKE, None) == -1
    assert r(ok, 3, FAKE, None) == -1
    assert r(ok, 1, None, None) == -2
    assert r(ok, 2, _at(FAKE, 8), None) == -1  # misaligned


def test_layout_and_switch_validation(L_):
    assert L_.sym_pack(_dims(4, 4, 4, 5), 1, FAKE, FAKE, None) == -1
    assert L_.sym_pack(_dims(4, 4, 4, 4), 1, None, FAKE, None) == -2
    assert L_.sym_unpack(_dims(4, 4, 4, 4), 0, FAKE, FAKE, None) == -1
    assert L_.sym_set_force_algorithm(3) == -1
    assert L_.sym_set_force_algorithm(0) == 0
    bad = (ctypes.c_double * 3)(1.0, math.nan, 0.0)
    assert L_.sym_set_coeffs_override(bad) == -1
    assert L_.sym_set_coeffs_override(None) == 0
    for s in (0, -1, -2, -3, -4, -5, 99):
        assert len(L_.sym_strerror(s)) > 0


def test_fat_validation(L_):
    ok = _dims(4, 4, 4, 4)
    c = (ctypes.c_double * 6)(5 / 8, -1 / 16, 1 / 64, -1 / 384, -1 / 16, -1 / 24)
    # 19 link fields of intermediates
    n32 = L_.sym_fat_workspace_bytes(ok, 1)
    assert n32 >= 19 * 4 * 256 * 9 * 8
    assert L_.sym_fat_workspace_bytes(ok, 2) >= 2 * 19 * 4 * 256 * 9 * 8
    assert L_.sym_fat_workspace_bytes(_dims(4, 4, 4, 3), 1) == 0
    fl = L_.sym_fat_links
    assert fl(ok, 1, None, FAKE, FAKE2, None, FAKE3, HUGE, None) == -2
    bad = (ctypes.c_double * 6)(1, 0, 0, math.inf, 0, 0)
    assert fl(ok, 1, bad, FAKE, FAKE2, None, FAKE3, HUGE, None) == -1
    assert fl(ok, 1, c, FAKE, None, None, FAKE3, HUGE, None) == -2
    assert fl(ok, 1, c, FAKE, FAKE2, MISALIGNED, FAKE3, HUGE, None) == -1
    assert fl(ok, 1, c, FAKE, FAKE2, None, FAKE3, 64, None) == -3
    assert fl(ok, 1, c, FAKE, FAKE, None, FAKE3, HUGE, None) == -1     # V == U
    assert fl(ok, 1, c, FAKE, FAKE2, FAKE2, FAKE3, HUGE, None) == -1   # W == V
    ff = L_.sym_fat_force
    assert ff(ok, 1, c, FAKE, FAKE2, None, FAKE4, 4, FAKE3, HUGE, None) == -1   # mode
    assert ff(ok, 1, c, FAKE, FAKE2, None, FAKE4, -1, FAKE3, HUGE, None) == -1
    assert ff(ok, 1, c, FAKE, None, None, FAKE4, 0, FAKE3, HUGE, None) == -2   # GV required
    assert ff(ok, 1, c, FAKE, FAKE2, None, None, 0, FAKE3, HUGE, None) == -2   # out required
    assert ff(ok, 3, c, FAKE, FAKE2, None, FAKE4, 0, FAKE3, HUGE, None) == -1
    assert ff(ok, 2, c, FAKE, FAKE2, FAKE2, FAKE4, 1, FAKE3, 8, None) == -3
    assert ff(ok, 1, c, FAKE, FAKE2, None, FAKE2, 0, FAKE3, HUGE, None) == -1  # out == GV


def test_wilson_validation(L_):
    ok = _dims(4, 4, 4, 4)
    assert L_.sym_wilson_workspace_bytes(ok, 1) >= 2 * 6 * 9 * 128 * 4
    assert L_.sym_wilson_workspace_bytes(_dims(4, 4, 5, 4), 1) == 0
    w = L_.sym_wilson_force
    X, Y = ctypes.c_void_p(0x14000000), ctypes.c_void_p(0x15000000)
    assert w(ok, 1, math.nan, 1.0, FAKE, X, Y, FAKE2, FAKE3, HUGE, None) == -1
    assert w(ok, 1, 0.12, math.inf, FAKE, X, Y, FAKE2, FAKE3, HUGE, None) == -1
    assert w(ok, 1, 0.12, 1.0, FAKE, None, Y, FAKE2, FAKE3, HUGE, None) == -2
    assert w(ok, 1, 0.12, 1.0, FAKE, X, Y, MISALIGNED, FAKE3, HUGE, None) == -1
    assert w(ok, 1, 0.12, 1.0, FAKE, X, Y, FAKE2, FAKE3, 16, None) == -3
    assert w(ok, 1, 0.12, 1.0, FAKE, X, Y, X, FAKE3, HUGE, None) == -1   # G == X
    assert L_.sym_pack_spinor(_dims(4, 4, 4, 3), 1, FAKE, FAKE2, None) == -1
    assert L_.sym_unpack_spinor(ok, 1, None, FAKE2, None) == -2


def test_probe_library_is_separate(L_):
    """The benchmark's FMA-rate probe lives in libsymprobe.so, outside the libsym ABI."""
    assert not hasattr(L_, "sym_fma_probe")
    path = os.path.join(ROOT, "paper_1808_02281_amd", "libsymprobe.so")
    P = ctypes.CDLL(path)
    P.probe_fma.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert P.probe_fma(3, 16, FAKE, None) == -1
    assert P.probe_fma(1, 0, FAKE, None) == -1
    assert P.probe_fma(1, (1 << 20) + 1, FAKE, None) == -1
    assert P.probe_fma(1, 16, MISALIGNED, None) == -1
    assert P.probe_fma(2, 16, None, None) == -2


def test_batch_validation(L_):
    """Every call below is rejected before anything is launched."""
    two = (ctypes.c_int32 * 8)(4, 4, 4, 4, 6, 6, 6, 8)
    bad = (ctypes.c_int32 * 8)(4, 4, 4, 4, 6, 6, 5, 8)
    ptrs = (ctypes.c_void_p * 2)(0x10000000, 0x11000000)
    outs = (ctypes.c_void_p * 2)(0x12000000, 0x13000000)
    holes = (ctypes.c_void_p * 2)(0x10000000, None)
    WS = ctypes.c_void_p(0x20000000)
    wb = L_.sym_batch_workspace_bytes
    assert wb(2, two, 1) > 0 and wb(2, two, 2) > wb(2, two, 1)
    assert wb(0, two, 1) == 0 and wb(2, bad, 1) == 0 and wb(2, None, 1) == 0 and wb(2, two, 3) == 0
    fb = L_.sym_force_batch
    assert fb(0, two, 0.8677, 3.0, 1, ptrs, outs, None, WS, HUGE, None) == -1
    assert fb(2, bad, 0.8677, 3.0, 1, ptrs, outs, None, WS, HUGE, None) == -1
    assert fb(2, None, 0.8677, 3.0, 1, ptrs, outs, None, WS, HUGE, None) == -2
    assert fb(2, two, -1.0, 3.0, 1, ptrs, outs, None, WS, HUGE, None) == -1
    assert fb(2, two, 0.8677, 3.0, 1, holes, outs, None, WS, HUGE, None) == -2
    assert fb(2, two, 0.8677, 3.0, 1, ptrs, None, None, WS, HUGE, None) == -2
    assert fb(2, two, 0.8677, 3.0, 1, ptrs, outs, MISALIGNED, WS, HUGE, None) == -1
    assert fb(2, two, 0.8677, 3.0, 1, ptrs, outs, None, None, HUGE, None) == -2
    assert fb(2, two, 0.8677, 3.0, 1, ptrs, outs, None, WS, 64, None) == -3
    at = L_.sym_batch_autotune
    assert at(0, two, 0.8677, 3.0, 1, ptrs, outs, WS, HUGE, None, None, 0, None, None, None) == -1
    assert at(2, two, 0.8677, 3.0, 2, holes, outs, WS, HUGE, None, None, 0, None, None, None) == -2
    assert at(2, two, 0.8677, 3.0, 1, ptrs, outs, WS, 64, None, None, 0, None, None, None) == -3
    # an output aliasing an input of another lattice, or two outputs coinciding
    assert fb(2, two, 0.8677, 3.0, 1, ptrs, ptrs, None, WS, HUGE, None) == -1
    crossed = (ctypes.c_void_p * 2)(0x12000000, 0x10000000)
    assert fb(2, two, 0.8677, 3.0, 1, ptrs, crossed, None, WS, HUGE, None) == -1
    same = (ctypes.c_void_p * 2)(0x12000000, 0x12000000)
    assert fb(2, two, 0.8677, 3.0, 1, ptrs, same, None, WS, HUGE, None) == -1
    assert at(2, two, 0.8677, 3.0, 1, ptrs, same, WS, HUGE, None, None, 0, None, None, None) == -1
    assert at(2, two, 0.8677, 3.0, 1, ptrs, outs, WS, HUGE, None, None, -1, None, None, None) == -1   # max_log


def test_static_force_validation(L_):
    """sym_force_static (no workspace argument) validates like sym_force and rejects a
    lattice whose workspace exceeds its fixed 64 MiB array before touching the device."""
    ok = _dims(4, 4, 4, 4)
    f = L_.sym_force_static
    assert f(_dims(4, 4, 3, 4), 0.8677, 3.0, 1, FAKE, FAKE2, None, None) == -1
    assert f(None, 0.8677, 3.0, 1, FAKE, FAKE2, None, None) == -2
    assert f(ok, 0.8677, 3.0, 7, FAKE, FAKE2, None, None) == -1
    assert f(ok, 0.0, 3.0, 1, FAKE, FAKE2, None, None) == -1
    assert f(ok, 0.8677, 3.0, 1, None, FAKE2, None, None) == -2
    assert f(ok, 0.8677, 3.0, 1, FAKE, None, None, None) == -2
    assert f(ok, 0.8677, 3.0, 1, FAKE, FAKE2, MISALIGNED, None) == -1
    assert f(_dims(16, 16, 16, 16), 0.8677, 3.0, 1, FAKE, FAKE2, None, None) == -3
    assert f(_dims(14, 14, 14, 14), 0.8677, 3.0, 2, FAKE, FAKE2, None, None) == -3
    assert L_.sym_workspace_bytes(_dims(14, 14, 14, 14), 1) <= 64 << 20
    assert L_.sym_workspace_bytes(_dims(12, 12, 12, 12), 2) <= 64 << 20
