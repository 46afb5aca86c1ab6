"""Python binding over the C ABI (include/sym.h): argument marshalling only.

Fields live on the GPU as torch tensors in the even-odd structure-of-arrays layout:
real tensors of shape ``(4, 2, 9, V/2, 2)`` (direction, parity, matrix element,
checkerboard site, re/im), float32 or float64. Every computation runs in the HIP
kernels of libsym.so on the current torch stream; nothing here computes physics.
"""
import ctypes

import torch

from . import _lib

_WS_CACHE = {}


def prec_of(dtype):
    if dtype == torch.float32:
        return _lib.SYM_F32
    if dtype == torch.float64:
        return _lib.SYM_F64
    raise TypeError(f"fields must be float32 or float64, got {dtype}")


def volume(L):
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return Lx * Ly * Lz * Lt


def field_shape(L):
    """Shape of a link/force/momentum field in the SoA even-odd layout."""
    return (4, 2, 9, volume(L) // 2, 2)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_field(name, t, L):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != field_shape(L):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {field_shape(L)} for L={tuple(L)}")
    prec_of(t.dtype)


def coeffs(u0):
    """(c_plaq, c_rect, c_cube), alpha_s (host computation inside the library)."""
    c = (ctypes.c_double * 3)()
    a = ctypes.c_double()
    _lib.check("sym_coeffs", _lib.lib().sym_coeffs(float(u0), c, ctypes.byref(a)))
    return [c[0], c[1], c[2]], a.value


def workspace_bytes(L, prec):
    return int(_lib.lib().sym_workspace_bytes(_lib.dims(L), int(prec)))


def workspace(L, prec, device):
    """A cached device workspace of sym_workspace_bytes(L, prec) bytes."""
    device = torch.device(device)
    key = (device.index, tuple(int(v) for v in L), int(prec))
    ws = _WS_CACHE.get(key)
    if ws is None:
        n = workspace_bytes(L, prec)
        if n == 0:
            raise ValueError(f"invalid lattice {tuple(L)} or precision {prec}")
        ws = torch.empty(n, dtype=torch.uint8, device=device)
        _WS_CACHE[key] = ws
    return ws


def release_workspaces():
    _WS_CACHE.clear()


def pack(aos, L):
    """Canonical complex (Lt,Lz,Ly,Lx,4,3,3) CUDA tensor -> SoA even-odd real field."""
    if not aos.is_cuda or not aos.is_contiguous():
        raise ValueError("aos must be a contiguous CUDA tensor")
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    if tuple(aos.shape) != (Lt, Lz, Ly, Lx, 4, 3, 3):
        raise ValueError(f"aos shape {tuple(aos.shape)} does not match L={tuple(L)}")
    real = {torch.complex64: torch.float32, torch.complex128: torch.float64}.get(aos.dtype)
    if real is None:
        raise TypeError("aos must be complex64 or complex128")
    out = torch.empty(field_shape(L), dtype=real, device=aos.device)
    _lib.check("sym_pack", _lib.lib().sym_pack(_lib.dims(L), prec_of(real), _ptr(aos), _ptr(out), _stream(aos.device)))
    return out


def unpack(soa, L):
    """SoA even-odd real field -> canonical complex (Lt,Lz,Ly,Lx,4,3,3) tensor."""
    _check_field("soa", soa, L)
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    cdt = torch.complex64 if soa.dtype == torch.float32 else torch.complex128
    out = torch.empty((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=cdt, device=soa.device)
    _lib.check("sym_unpack", _lib.lib().sym_unpack(_lib.dims(L), prec_of(soa.dtype), _ptr(soa), _ptr(out),
                                                   _stream(soa.device)))
    return out


def action(U, L, u0, beta):
    """S_G and W_P, W_R, W_C as a float64 CUDA tensor of 4 (asynchronous)."""
    _check_field("U", U, L)
    prec = prec_of(U.dtype)
    ws = workspace(L, prec, U.device)
    S = torch.empty(4, dtype=torch.float64, device=U.device)
    _lib.check("sym_action", _lib.lib().sym_action(_lib.dims(L), float(u0), float(beta), prec, _ptr(U), _ptr(S),
                                                   _ptr(ws), ws.numel(), _stream(U.device)))
    return S


def force(U, L, u0, beta, with_action=False, out=None):
    """G = (beta/6)(U t)_TA on every link; with_action also returns S as in ``action``."""
    _check_field("U", U, L)
    prec = prec_of(U.dtype)
    ws = workspace(L, prec, U.device)
    F = torch.empty_like(U) if out is None else out
    _check_field("out", F, L)
    S = torch.empty(4, dtype=torch.float64, device=U.device) if with_action else None
    _lib.check("sym_force", _lib.lib().sym_force(_lib.dims(L), float(u0), float(beta), prec, _ptr(U), _ptr(F),
                                                 _ptr(S) if S is not None else None, _ptr(ws), ws.numel(),
                                                 _stream(U.device)))
    return (F, S) if with_action else F


def action_grad(U, L, u0, beta, with_action=False):
    """2 G U on every link: dS_G/dU projected on the tangent space of SU(3) at U."""
    _check_field("U", U, L)
    prec = prec_of(U.dtype)
    ws = workspace(L, prec, U.device)
    gr = torch.empty_like(U)
    S = torch.empty(4, dtype=torch.float64, device=U.device) if with_action else None
    _lib.check("sym_action_grad", _lib.lib().sym_action_grad(_lib.dims(L), float(u0), float(beta), prec, _ptr(U),
                                                             _ptr(gr), _ptr(S) if S is not None else None,
                                                             _ptr(ws), ws.numel(), _stream(U.device)))
    return (gr, S) if with_action else gr


def md_leapfrog(U, P, L, u0, beta, dt, nsteps, with_energy=True):
    """In-place leapfrog on (U, P); returns H = [H_start, H_end] (float64 CUDA tensor)."""
    _check_field("U", U, L)
    _check_field("P", P, L)
    if U.dtype != P.dtype:
        raise TypeError("U and P must have the same dtype")
    prec = prec_of(U.dtype)
    ws = workspace(L, prec, U.device)
    H = torch.empty(2, dtype=torch.float64, device=U.device) if with_energy else None
    _lib.check("md_leapfrog", _lib.lib().md_leapfrog(_lib.dims(L), float(u0), float(beta), prec, _ptr(U), _ptr(P),
                                                     float(dt), int(nsteps), _ptr(H) if H is not None else None,
                                                     _ptr(ws), ws.numel(), _stream(U.device)))
    return H


def check_links(U, L):
    """{max ||U^+U - 1||_F, max |det U - 1|, non-finite links} of a link field as a float64
    CUDA tensor of 3 (asynchronous; sym_check_links)."""
    _check_field("U", U, L)
    prec = prec_of(U.dtype)
    ws = workspace(L, prec, U.device)
    out = torch.empty(3, dtype=torch.float64, device=U.device)
    _lib.check("sym_check_links", _lib.lib().sym_check_links(_lib.dims(L), prec, _ptr(U), _ptr(out), _ptr(ws),
                                                             ws.numel(), _stream(U.device)))
    return out


def reunitarise(U, L):
    """Project every link of U onto SU(3) in place (sym_reunitarise); returns U."""
    _check_field("U", U, L)
    _lib.check("sym_reunitarise", _lib.lib().sym_reunitarise(_lib.dims(L), prec_of(U.dtype), _ptr(U),
                                                             _stream(U.device)))
    return U


def set_coeffs_override(c):
    """Use loop coefficients c = (c_plaq, c_rect, c_cube) instead of u0's; None restores."""
    if c is None:
        return _lib.check("sym_set_coeffs_override", _lib.lib().sym_set_coeffs_override(None))
    arr = (ctypes.c_double * 3)(*[float(v) for v in c])
    return _lib.check("sym_set_coeffs_override", _lib.lib().sym_set_coeffs_override(arr))


def set_force_algorithm(name):
    """'auto' (default), 'direct' or 'factored'."""
    return _lib.check("sym_set_force_algorithm", _lib.lib().sym_set_force_algorithm(_lib.ALGORITHMS[name]))


def profile_enable(on=True):
    """Bracket every library kernel launch with HIP timing events (see sym_profile_enable)."""
    return _lib.check("sym_profile_enable", _lib.lib().sym_profile_enable(1 if on else 0))


def profile_collect(max_kinds=32):
    """{kernel name: (total ms, launches)} for the launches recorded since the last call."""
    names = ctypes.create_string_buffer(32 * max_kinds)
    ms = (ctypes.c_double * max_kinds)()
    cnt = (ctypes.c_int32 * max_kinds)()
    n = _lib.lib().sym_profile_collect(max_kinds, names, ms, cnt)
    if n < 0:
        _lib.check("sym_profile_collect", n)
    raw = names.raw
    out = {}
    for k in range(n):
        name = raw[32 * k: 32 * k + 32].split(b"\0", 1)[0].decode()
        out[name] = (ms[k], cnt[k])
    return out


def _batch_args(Us, Ls):
    n = len(Us)
    if n == 0 or len(Ls) != n:
        raise ValueError("need one lattice shape per field")
    for i, (U, L) in enumerate(zip(Us, Ls)):
        _check_field(f"U[{i}]", U, L)
        if U.dtype != Us[0].dtype or U.device != Us[0].device:
            raise ValueError("all fields of a batch must share dtype and device")
    Lflat = (ctypes.c_int32 * (4 * n))(*[int(v) for L in Ls for v in L])
    return n, Lflat, prec_of(Us[0].dtype)


def batch_workspace(Ls, prec, device):
    device = torch.device(device)
    key = ("batch", device.index, tuple(tuple(int(v) for v in L) for L in Ls), int(prec))
    ws = _WS_CACHE.get(key)
    if ws is None:
        n = len(Ls)
        Lflat = (ctypes.c_int32 * (4 * n))(*[int(v) for L in Ls for v in L])
        nb = int(_lib.lib().sym_batch_workspace_bytes(n, Lflat, int(prec)))
        if nb == 0:
            raise ValueError("invalid batch")
        ws = torch.empty(nb, dtype=torch.uint8, device=device)
        _WS_CACHE[key] = ws
    return ws


def force_batch(Us, Ls, u0, beta, with_action=False, out=None, S_out=None):
    """Forces of many independent lattices in one launch per pass (sym_force_batch).

    Returns the list of force fields (``out`` if given) and, with_action, a float64
    (n, 4) tensor of S, W_P, W_R, W_C per lattice (``S_out`` if given)."""
    n, Lflat, prec = _batch_args(Us, Ls)
    dev = Us[0].device
    ws = batch_workspace(Ls, prec, dev)
    Fs = [torch.empty_like(U) for U in Us] if out is None else out
    for i, (F, L) in enumerate(zip(Fs, Ls)):
        _check_field(f"out[{i}]", F, L)
    S = None
    if with_action:
        S = torch.empty((n, 4), dtype=torch.float64, device=dev) if S_out is None else S_out
    Up = (ctypes.c_void_p * n)(*[U.data_ptr() for U in Us])
    Fp = (ctypes.c_void_p * n)(*[F.data_ptr() for F in Fs])
    _lib.check("sym_force_batch", _lib.lib().sym_force_batch(n, Lflat, float(u0), float(beta), prec, Up, Fp,
                                                             _ptr(S) if S is not None else None, _ptr(ws),
                                                             ws.numel(), _stream(dev)))
    return (Fs, S) if with_action else Fs


def batch_autotune(Us, Ls, u0, beta, out=None):
    """Time the candidate schedules of force_batch for this batch (sym_batch_autotune);
    the best one is kept for later force_batch calls with the same lattice shapes.
    Returns (best, log): best = {grid, order, links, lds_kib} (grid 0 is one workgroup per
    tile, lds_kib -1 the default occupancy), log = [(schedule dict, ms per batch), ...]
    for every candidate. ``out`` (optional, one field per lattice) receives the forces of
    the last schedule timed."""
    n, Lflat, prec = _batch_args(Us, Ls)
    dev = Us[0].device
    ws = batch_workspace(Ls, prec, dev)
    Fs = [torch.empty_like(U) for U in Us] if out is None else out
    if len(Fs) != n:
        raise ValueError("out needs one field per lattice")
    for U, F in zip(Us, Fs):
        if F.shape != U.shape or F.dtype != U.dtype or not F.is_contiguous():
            raise ValueError("out fields must match U in shape and dtype and be contiguous")
    Up = (ctypes.c_void_p * n)(*[U.data_ptr() for U in Us])
    Fp = (ctypes.c_void_p * n)(*[F.data_ptr() for F in Fs])
    best = (ctypes.c_int32 * 4)()
    nmax = 256
    sched = (ctypes.c_int32 * (4 * nmax))()
    ms = (ctypes.c_float * nmax)()
    nlog = ctypes.c_int32()
    _lib.check("sym_batch_autotune", _lib.lib().sym_batch_autotune(n, Lflat, float(u0), float(beta), prec, Up, Fp,
                                                                   _ptr(ws), ws.numel(), _stream(dev), best, nmax,
                                                                   sched, ms, ctypes.byref(nlog)))
    keys = ("grid", "order", "links", "lds_kib")
    as_dict = lambda v: {k: int(x) for k, x in zip(keys, v)}
    log = [(as_dict(sched[4 * i: 4 * i + 4]), float(ms[i])) for i in range(nlog.value)]
    return as_dict(best[:]), log


# ------------------------------------------------------------------ fat links

def _fat_c(c):
    c = [float(v) for v in c]
    if len(c) != 6:
        raise ValueError("fat-link coefficients are (c_1, c_3, c_5, c_7, c_L, c_N)")
    return (ctypes.c_double * 6)(*c)


def fat_workspace(L, prec, device):
    """A cached device workspace of sym_fat_workspace_bytes(L, prec) bytes."""
    device = torch.device(device)
    key = ("fat", device.index, tuple(int(v) for v in L), int(prec))
    ws = _WS_CACHE.get(key)
    if ws is None:
        n = int(_lib.lib().sym_fat_workspace_bytes(_lib.dims(L), int(prec)))
        if n == 0:
            raise ValueError(f"invalid lattice {tuple(L)} or precision {prec}")
        ws = torch.empty(n, dtype=torch.uint8, device=device)
        _WS_CACHE[key] = ws
    return ws


def new_fat_workspace(L, prec, device):
    """A private (uncached) fat-link workspace, for keeping forward intermediates."""
    n = int(_lib.lib().sym_fat_workspace_bytes(_lib.dims(L), int(prec)))
    if n == 0:
        raise ValueError(f"invalid lattice {tuple(L)} or precision {prec}")
    return torch.empty(n, dtype=torch.uint8, device=torch.device(device))


def _check_ws(ws, L, prec, device):
    n = int(_lib.lib().sym_fat_workspace_bytes(_lib.dims(L), int(prec)))
    if ws.dtype != torch.uint8 or ws.numel() < n or ws.device != torch.device(device) or not ws.is_contiguous():
        raise ValueError("ws must be a contiguous uint8 device tensor of sym_fat_workspace_bytes bytes")


def fat_links(U, L, c, with_naik=True, out=None, ws=None):
    """Asqtad/HISQ fat links V (and Naik links W) of a link field (sym_fat_links).

    c = (c_1, c_3, c_5, c_7, c_L, c_N). Returns V, or (V, W) with_naik; ``out`` may
    give V or (V, W). ``ws``: a workspace to use instead of the cached one (it then
    holds the forward intermediates for fat_force(..., reuse_links=True))."""
    _check_field("U", U, L)
    prec = prec_of(U.dtype)
    if ws is None:
        ws = fat_workspace(L, prec, U.device)
    else:
        _check_ws(ws, L, prec, U.device)
    if out is None:
        V = torch.empty_like(U)
        W = torch.empty_like(U) if with_naik else None
    else:
        V, W = (out if with_naik else (out, None))
    _check_field("V", V, L)
    if W is not None:
        _check_field("W", W, L)
    _lib.check("sym_fat_links", _lib.lib().sym_fat_links(_lib.dims(L), prec, _fat_c(c), _ptr(U), _ptr(V),
                                                         _ptr(W) if W is not None else None, _ptr(ws), ws.numel(),
                                                         _stream(U.device)))
    return (V, W) if with_naik else V


def fat_force(U, L, c, GV, GW=None, mode="grad", out=None, ws=None, reuse_links=False):
    """Pull-back of the adjoint fields GV (of V) and GW (of W, optional) to the thin links
    (sym_fat_force): mode 'grad' gives dPhi/dRe U + i dPhi/dIm U, 'force' the traceless
    antihermitian G = -(1/2)(U grad^+)_TA (gauge-force convention). ``reuse_links``:
    ``ws`` holds the intermediates of fat_links(U, L, c, ws=ws), so the forward passes
    are skipped."""
    _check_field("U", U, L)
    _check_field("GV", GV, L)
    if GW is not None:
        _check_field("GW", GW, L)
    for t in (GV, GW):
        if t is not None and t.dtype != U.dtype:
            raise TypeError("adjoint fields must have the dtype of U")
    prec = prec_of(U.dtype)
    if reuse_links and ws is None:
        raise ValueError("reuse_links needs the workspace that fat_links filled")
    if ws is None:
        ws = fat_workspace(L, prec, U.device)
    else:
        _check_ws(ws, L, prec, U.device)
    o = torch.empty_like(U) if out is None else out
    _check_field("out", o, L)
    m = _lib.FAT_MODES[mode] | (_lib.FAT_REUSE_LINKS if reuse_links else 0)
    _lib.check("sym_fat_force", _lib.lib().sym_fat_force(_lib.dims(L), prec, _fat_c(c), _ptr(U), _ptr(GV),
                                                         _ptr(GW) if GW is not None else None, _ptr(o), m,
                                                         _ptr(ws), ws.numel(), _stream(U.device)))
    return o


# ----------------------------------------------------------- Wilson-clover force

def spinor_shape(L):
    """Shape of a spinor field in the SoA even-odd layout: (2, 12, V/2, 2) reals."""
    return (2, 12, volume(L) // 2, 2)


def _check_spinor(name, t, L):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA (HIP) tensor")
    if tuple(t.shape) != spinor_shape(L):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {spinor_shape(L)} for L={tuple(L)}")
    prec_of(t.dtype)


def pack_spinor(aos, L):
    """Canonical complex (Lt,Lz,Ly,Lx,4,3) CUDA tensor -> SoA even-odd spinor field."""
    if not aos.is_cuda or not aos.is_contiguous():
        raise ValueError("aos must be a contiguous CUDA tensor")
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    if tuple(aos.shape) != (Lt, Lz, Ly, Lx, 4, 3):
        raise ValueError(f"aos shape {tuple(aos.shape)} does not match L={tuple(L)}")
    real = {torch.complex64: torch.float32, torch.complex128: torch.float64}.get(aos.dtype)
    if real is None:
        raise TypeError("aos must be complex64 or complex128")
    out = torch.empty(spinor_shape(L), dtype=real, device=aos.device)
    _lib.check("sym_pack_spinor", _lib.lib().sym_pack_spinor(_lib.dims(L), prec_of(real), _ptr(aos), _ptr(out),
                                                             _stream(aos.device)))
    return out


def unpack_spinor(soa, L):
    """SoA even-odd spinor field -> canonical complex (Lt,Lz,Ly,Lx,4,3) tensor."""
    _check_spinor("soa", soa, L)
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    cdt = torch.complex64 if soa.dtype == torch.float32 else torch.complex128
    out = torch.empty((Lt, Lz, Ly, Lx, 4, 3), dtype=cdt, device=soa.device)
    _lib.check("sym_unpack_spinor", _lib.lib().sym_unpack_spinor(_lib.dims(L), prec_of(soa.dtype), _ptr(soa),
                                                                 _ptr(out), _stream(soa.device)))
    return out


def wilson_workspace(L, prec, device):
    device = torch.device(device)
    key = ("wilson", device.index, tuple(int(v) for v in L), int(prec))
    ws = _WS_CACHE.get(key)
    if ws is None:
        n = int(_lib.lib().sym_wilson_workspace_bytes(_lib.dims(L), int(prec)))
        if n == 0:
            raise ValueError(f"invalid lattice {tuple(L)} or precision {prec}")
        ws = torch.empty(n, dtype=torch.uint8, device=device)
        _WS_CACHE[key] = ws
    return ws


def wilson_force(U, X, Y, L, kappa, csw, out=None):
    """G with dPsi/domega^a = -2i tr(T_a G), Psi = Y^+ D X + c.c. (sym_wilson_force)."""
    _check_field("U", U, L)
    _check_spinor("X", X, L)
    _check_spinor("Y", Y, L)
    if X.dtype != U.dtype or Y.dtype != U.dtype:
        raise TypeError("X and Y must have the dtype of U")
    prec = prec_of(U.dtype)
    ws = wilson_workspace(L, prec, U.device)
    G = torch.empty_like(U) if out is None else out
    _check_field("out", G, L)
    _lib.check("sym_wilson_force", _lib.lib().sym_wilson_force(_lib.dims(L), prec, float(kappa), float(csw), _ptr(U),
                                                               _ptr(X), _ptr(Y), _ptr(G), _ptr(ws), ws.numel(),
                                                               _stream(U.device)))
    return G
