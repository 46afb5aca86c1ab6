"""sym_force_static, the entry point for callers that cannot allocate: called through
the C ABI, its forces and actions equal sym_force's (same kernels, same algorithm) on two
calls in a row, the second on a smaller lattice, and a lattice too large for its fixed
scratch array is rejected with SYM_EWORKSPACE before anything is launched."""
import ctypes

import numpy as np
import pytest
import torch

import gaugegen

from gpu_util import device, to_soa

pytestmark = pytest.mark.gpu

U0, BETA = gaugegen.U0, gaugegen.BETA


def _static_force(sym, lib, Us, L):
    from paper_1808_02281_amd import _lib

    F = torch.empty_like(Us)
    S = torch.empty(4, dtype=torch.float64, device=Us.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream(Us.device).cuda_stream)
    rc = lib.sym_force_static(_lib.dims(L), U0, BETA, sym.prec_of(Us.dtype), ctypes.c_void_p(Us.data_ptr()),
                              ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(S.data_ptr()), stream)
    assert rc == 0, lib.sym_strerror(rc)
    return F, S


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_static_force_matches_sym_force(prec):
    import paper_1808_02281_amd as sym
    from paper_1808_02281_amd import _lib

    lib = _lib.lib()
    dev = device()
    sym.set_force_algorithm("auto")
    for L, seed in (((8, 8, 8, 8), 41), ((6, 4, 6, 8), 42)):   # the second call is smaller
        print(f"case sym_force_static {prec} L={L}", flush=True)
        Us = to_soa(sym, gaugegen.near_thermal_links(L, 0.3, seed), L, prec, dev)
        Fs, Ss = _static_force(sym, lib, Us, L)
        F, S = sym.force(Us, L, U0, BETA, with_action=True)
        torch.cuda.synchronize()
        tol = 1e-12 if prec == "f64" else 1e-5
        df = (torch.abs(Fs - F).max() / torch.abs(F).max()).item()
        ds = np.abs(Ss.cpu().numpy() - S.cpu().numpy()) / np.abs(S.cpu().numpy())
        print(f"  force {df:.2e}, action and W {ds.max():.2e}", flush=True)
        assert df <= tol and ds.max() <= tol


def test_static_force_rejects_large_lattices():
    import paper_1808_02281_amd as sym
    from paper_1808_02281_amd import _lib

    lib = _lib.lib()
    dev = device()
    L = (16, 16, 16, 16)                 # 201 MB of FP64 workspace, beyond the 64 MiB array
    Us = torch.empty(sym.field_shape(L), dtype=torch.float64, device=dev)
    F = torch.empty_like(Us)
    rc = lib.sym_force_static(_lib.dims(L), U0, BETA, 2, ctypes.c_void_p(Us.data_ptr()),
                              ctypes.c_void_p(F.data_ptr()), None, None)
    assert rc == -3
