"""ctypes wrapper over ``libsymoracle.so`` (FP64 C oracle). Test infrastructure only.

Arrays are numpy complex128 in the canonical array-of-structures lexicographic layout
``(Lt, Lz, Ly, Lx, 4, 3, 3)``: site index ``((t*Lz + z)*Ly + y)*Lx + x``, direction
``mu = 0..3`` for ``x, y, z, t``. ``L`` is always given as ``(Lx, Ly, Lz, Lt)``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsymoracle.so")
_lib = None

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int32_p = ctypes.POINTER(ctypes.c_int32)
_c_int64_p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build

        build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.orc_coeffs.argtypes = [ctypes.c_double, _c_double_p, _c_double_p]
    lib.orc_coeffs.restype = ctypes.c_int
    lib.orc_loop_table.argtypes = [_c_int32_p, _c_int32_p, _c_int32_p]
    lib.orc_loop_table.restype = ctypes.c_int
    lib.orc_action.argtypes = [_c_int32_p, _c_double_p, ctypes.c_double, vp, _c_double_p]
    lib.orc_action.restype = ctypes.c_double
    lib.orc_force.argtypes = [_c_int32_p, _c_double_p, ctypes.c_double, vp, vp]
    lib.orc_force.restype = None
    lib.orc_force_links.argtypes = [_c_int32_p, _c_double_p, ctypes.c_double, vp, ctypes.c_int64,
                                    _c_int64_p, _c_int32_p, vp]
    lib.orc_force_links.restype = None
    lib.orc_staple_sums.argtypes = [_c_int32_p, vp, vp]
    lib.orc_staple_sums.restype = None
    lib.orc_local_action.argtypes = [_c_int32_p, _c_double_p, ctypes.c_double, vp, ctypes.c_int64,
                                     ctypes.c_int32]
    lib.orc_local_action.restype = ctypes.c_double
    lib.orc_su3_exp.argtypes = [ctypes.c_int64, vp, vp]
    lib.orc_su3_exp.restype = None
    lib.orc_kinetic.argtypes = [_c_int32_p, vp]
    lib.orc_kinetic.restype = ctypes.c_double
    lib.orc_leapfrog.argtypes = [_c_int32_p, _c_double_p, ctypes.c_double, vp, vp, ctypes.c_double,
                                 ctypes.c_int32, _c_double_p]
    lib.orc_leapfrog.restype = ctypes.c_int
    lib.orc_fat_paths.argtypes = [ctypes.c_int32, _c_int32_p, _c_int32_p, _c_int32_p]
    lib.orc_fat_paths.restype = ctypes.c_int
    lib.orc_fat_links.argtypes = [_c_int32_p, _c_double_p, vp, vp, vp]
    lib.orc_fat_links.restype = None
    lib.orc_fat_links_links.argtypes = [_c_int32_p, _c_double_p, vp, ctypes.c_int64, _c_int64_p, _c_int32_p, vp, vp]
    lib.orc_fat_links_links.restype = None
    lib.orc_fat_grad.argtypes = [_c_int32_p, _c_double_p, vp, vp, vp, vp]
    lib.orc_fat_grad.restype = None
    lib.orc_fat_grad_links.argtypes = [_c_int32_p, _c_double_p, vp, vp, vp, ctypes.c_int64, _c_int64_p,
                                       _c_int32_p, vp]
    lib.orc_fat_grad_links.restype = None
    lib.orc_fat_force_from_grad.argtypes = [ctypes.c_int64, vp, vp, vp]
    lib.orc_fat_force_from_grad.restype = None
    lib.orc_gamma.argtypes = [ctypes.c_int32, vp]
    lib.orc_gamma.restype = None
    lib.orc_clover_leaves.argtypes = [_c_int32_p, vp, vp]
    lib.orc_clover_leaves.restype = None
    lib.orc_wilson_apply.argtypes = [_c_int32_p, ctypes.c_double, ctypes.c_double, vp, vp, vp]
    lib.orc_wilson_apply.restype = None
    lib.orc_wilson_psi.argtypes = [_c_int32_p, ctypes.c_double, ctypes.c_double, vp, vp, vp]
    lib.orc_wilson_psi.restype = ctypes.c_double
    lib.orc_wilson_force.argtypes = [_c_int32_p, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp]
    lib.orc_wilson_force.restype = None
    lib.orc_wilson_force_links.argtypes = [_c_int32_p, ctypes.c_double, ctypes.c_double, vp, vp, vp, ctypes.c_int64,
                                           _c_int64_p, _c_int32_p, vp]
    lib.orc_wilson_force_links.restype = None
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _dims(L):
    a = (ctypes.c_int32 * 4)(*[int(v) for v in L])
    return a


def _cvec(c):
    return (ctypes.c_double * 3)(*[float(v) for v in c])


def _field(U, L):
    U = np.ascontiguousarray(U, dtype=np.complex128)
    Lx, Ly, Lz, Lt = L
    if U.shape != (Lt, Lz, Ly, Lx, 4, 3, 3):
        raise ValueError(f"field shape {U.shape} does not match L={tuple(L)}")
    return U


def coeffs(u0):
    """(c_plaq, c_rect, c_cube), alpha_s from u0 (eq. 18_3_27_30 and the alpha_s formula)."""
    c = (ctypes.c_double * 3)()
    a = ctypes.c_double()
    if _load().orc_coeffs(float(u0), c, ctypes.byref(a)) != 0:
        raise ValueError("u0 must be positive and finite")
    return np.array(list(c)), a.value


def loop_table():
    """The 34 loops: (len[34], cls[34], dirs[34,6]) with signed directions +-1..+-4."""
    ln = (ctypes.c_int32 * 34)()
    cl = (ctypes.c_int32 * 34)()
    d = (ctypes.c_int32 * (34 * 6))()
    n = _load().orc_loop_table(ln, cl, d)
    return np.array(ln[:n]), np.array(cl[:n]), np.array(d[:]).reshape(34, 6)[:n]


def action(U, L, c, beta):
    """S_G and W = (W_plaq, W_rect, W_cube) = per-class sums of Re tr P_n (eq. 18_6_4_1)."""
    U = _field(U, L)
    W = (ctypes.c_double * 3)()
    S = _load().orc_action(_dims(L), _cvec(c), float(beta), U.ctypes.data, W)
    return S, np.array(list(W))


def force(U, L, c, beta):
    """G = (beta/6)(U t)_TA on every link, shape like U (force algorithm of Sec. II)."""
    U = _field(U, L)
    G = np.empty_like(U)
    _load().orc_force(_dims(L), _cvec(c), float(beta), U.ctypes.data, G.ctypes.data)
    return G


def force_links(U, L, c, beta, sites, mus):
    """G on a list of links given by lexicographic site index and direction."""
    U = _field(U, L)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    mus = np.ascontiguousarray(mus, dtype=np.int32)
    G = np.empty((len(sites), 3, 3), dtype=np.complex128)
    _load().orc_force_links(_dims(L), _cvec(c), float(beta), U.ctypes.data, len(sites),
                            sites.ctypes.data_as(_c_int64_p), mus.ctypes.data_as(_c_int32_p),
                            G.ctypes.data)
    return G


def staple_sums(U, L):
    """Unweighted per-class staple sums t[cls] for every link: shape U.shape[:-2] + (3, 3, 3)."""
    U = _field(U, L)
    out = np.empty(U.shape[:-2] + (3, 3, 3), dtype=np.complex128)
    _load().orc_staple_sums(_dims(L), U.ctypes.data, out.ctypes.data)
    return out


def local_action(U, L, c, beta, site, mu):
    """The part of S_G carried by the loops through link (site, mu)."""
    U = _field(U, L)
    return _load().orc_local_action(_dims(L), _cvec(c), float(beta), U.ctypes.data, int(site), int(mu))


def su3_exp(X):
    """exp(X) for a stack of 3x3 complex matrices (Taylor series, scaling and squaring)."""
    X = np.ascontiguousarray(X, dtype=np.complex128)
    out = np.empty_like(X)
    n = X.size // 9
    _load().orc_su3_exp(n, X.ctypes.data, out.ctypes.data)
    return out


def kinetic(P, L):
    """sum over links of -tr(Pi^2) for antihermitian momenta Pi."""
    P = _field(P, L)
    return _load().orc_kinetic(_dims(L), P.ctypes.data)


def leapfrog(U, P, L, c, beta, dt, nsteps):
    """Leapfrog trajectory; returns (U_end, P_end, H_start, H_end). Inputs are not modified."""
    U = _field(U, L).copy()
    P = _field(P, L).copy()
    H = (ctypes.c_double * 2)()
    rc = _load().orc_leapfrog(_dims(L), _cvec(c), float(beta), U.ctypes.data, P.ctypes.data,
                              float(dt), int(nsteps), H)
    if rc != 0:
        raise MemoryError("oracle leapfrog could not allocate its force buffer")
    return U, P, H[0], H[1]


FAT_CLASSES = ("one-link", "three-staple", "five-staple", "seven-staple", "Lepage", "Naik")


def _c6(c):
    if len(c) != 6:
        raise ValueError("fat-link coefficients are (c_1, c_3, c_5, c_7, c_L, c_N)")
    return (ctypes.c_double * 6)(*[float(v) for v in c])


def fat_paths(mu):
    """Paths of the asqtad matrix for direction mu (0..3): (len[86], cls[86], dirs[86,7]).

    85 smearing paths from p to p+mu (eq. 18_6_6_7_2 and the Lepage term eq. 18_6_6_7),
    then the Naik path (eq. 18_6_6_3); classes index FAT_CLASSES; signed directions +-1..+-4.
    """
    ln = (ctypes.c_int32 * 86)()
    cl = (ctypes.c_int32 * 86)()
    d = (ctypes.c_int32 * (86 * 7))()
    n = _load().orc_fat_paths(int(mu), ln, cl, d)
    return np.array(ln[:n]), np.array(cl[:n]), np.array(d[:]).reshape(86, 7)[:n]


def fat_links(U, L, c):
    """(V, W): fat links and Naik long links (c_N included) of every link, shapes like U."""
    U = _field(U, L)
    V = np.empty_like(U)
    W = np.empty_like(U)
    _load().orc_fat_links(_dims(L), _c6(c), U.ctypes.data, V.ctypes.data, W.ctypes.data)
    return V, W


def fat_links_links(U, L, c, sites, mus):
    """(V, W) on a list of links (lexicographic site, direction): shapes (n, 3, 3)."""
    U = _field(U, L)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    mus = np.ascontiguousarray(mus, dtype=np.int32)
    V = np.empty((len(sites), 3, 3), dtype=np.complex128)
    W = np.empty_like(V)
    _load().orc_fat_links_links(_dims(L), _c6(c), U.ctypes.data, len(sites), sites.ctypes.data_as(_c_int64_p),
                                mus.ctypes.data_as(_c_int32_p), V.ctypes.data, W.ctypes.data)
    return V, W


def fat_grad(U, L, c, GV, GW=None):
    """grad of Phi = Re sum tr(GV^+ V) + Re sum tr(GW^+ W) w.r.t. U (dRe + i dIm), every link."""
    U = _field(U, L)
    GV = _field(GV, L)
    GWp = None if GW is None else _field(GW, L)
    out = np.empty_like(U)
    _load().orc_fat_grad(_dims(L), _c6(c), U.ctypes.data, GV.ctypes.data,
                         None if GWp is None else GWp.ctypes.data, out.ctypes.data)
    return out


def fat_grad_links(U, L, c, GV, GW, sites, mus):
    """fat_grad on a list of links (lexicographic site, direction): shape (n, 3, 3)."""
    U = _field(U, L)
    GV = _field(GV, L)
    GWp = None if GW is None else _field(GW, L)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    mus = np.ascontiguousarray(mus, dtype=np.int32)
    out = np.empty((len(sites), 3, 3), dtype=np.complex128)
    _load().orc_fat_grad_links(_dims(L), _c6(c), U.ctypes.data, GV.ctypes.data,
                               None if GWp is None else GWp.ctypes.data, len(sites),
                               sites.ctypes.data_as(_c_int64_p), mus.ctypes.data_as(_c_int32_p),
                               out.ctypes.data)
    return out


def fat_force_from_grad(U, grad):
    """G = -(1/2)(U grad^+)_TA per link (the gauge-force convention, eq. 18_7_24_6)."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    grad = np.ascontiguousarray(grad, dtype=np.complex128)
    if U.shape != grad.shape:
        raise ValueError("U and grad must have the same shape")
    G = np.empty_like(U)
    _load().orc_fat_force_from_grad(U.size // 9, U.ctypes.data, grad.ctypes.data, G.ctypes.data)
    return G


def _spinor(X, L):
    X = np.ascontiguousarray(X, dtype=np.complex128)
    Lx, Ly, Lz, Lt = L
    if X.shape != (Lt, Lz, Ly, Lx, 4, 3):
        raise ValueError(f"spinor shape {X.shape} does not match L={tuple(L)}")
    return X


def gamma(mu):
    """Hermitian gamma matrix gamma_{mu+1} (DeGrand-Rossi basis), mu = 0..3 for x, y, z, t."""
    g = np.empty((4, 4), dtype=np.complex128)
    _load().orc_gamma(int(mu), g.ctypes.data)
    return g


def clover_leaves(U, L):
    """Q_{n;mu nu} (eq. 17_7_20_8) for every site and ordered pair: shape (V, 4, 4, 3, 3)."""
    U = _field(U, L)
    V = int(np.prod(L))
    Q = np.empty((V, 4, 4, 3, 3), dtype=np.complex128)
    _load().orc_clover_leaves(_dims(L), U.ctypes.data, Q.ctypes.data)
    return Q


def wilson_apply(U, X, L, kappa, csw):
    """D X for the Wilson matrix with clover term (eqs. 18_7_17_2, 18_7_17_4, 18_7_18_0)."""
    U, X = _field(U, L), _spinor(X, L)
    out = np.empty_like(X)
    _load().orc_wilson_apply(_dims(L), float(kappa), float(csw), U.ctypes.data, X.ctypes.data, out.ctypes.data)
    return out


def wilson_psi(U, X, Y, L, kappa, csw):
    """Psi = Y^+ D X + c.c. = 2 Re Y^+ D X."""
    U, X, Y = _field(U, L), _spinor(X, L), _spinor(Y, L)
    return _load().orc_wilson_psi(_dims(L), float(kappa), float(csw), U.ctypes.data, X.ctypes.data, Y.ctypes.data)


def wilson_force(U, X, Y, L, kappa, csw):
    """G with dPsi/domega^a = -2i tr(T_a G) on every link (eqs. 18_6_24_0, 18_1_29_20_1, 18_7_17_31)."""
    U, X, Y = _field(U, L), _spinor(X, L), _spinor(Y, L)
    G = np.empty_like(U)
    _load().orc_wilson_force(_dims(L), float(kappa), float(csw), U.ctypes.data, X.ctypes.data, Y.ctypes.data,
                             G.ctypes.data)
    return G


def wilson_force_links(U, X, Y, L, kappa, csw, sites, mus):
    U, X, Y = _field(U, L), _spinor(X, L), _spinor(Y, L)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    mus = np.ascontiguousarray(mus, dtype=np.int32)
    G = np.empty((len(sites), 3, 3), dtype=np.complex128)
    _load().orc_wilson_force_links(_dims(L), float(kappa), float(csw), U.ctypes.data, X.ctypes.data,
                                   Y.ctypes.data, len(sites), sites.ctypes.data_as(_c_int64_p),
                                   mus.ctypes.data_as(_c_int32_p), G.ctypes.data)
    return G


def num_threads():
    return _load().orc_num_threads()


def set_num_threads(n):
    """OpenMP threads of the oracle's later calls from this thread; returns the count."""
    return _load().orc_set_num_threads(int(n))


def gell_mann():
    """T_a = lambda_a / 2, the su(3) generators with tr(T_a T_b) = delta_ab / 2 (eq. 18_1_29_3_0)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam / 2


def lie_derivative(G):
    """dS/domega^a = -2i tr(T_a G) for U -> exp(i omega.T) U (from the force identity of Sec. II)."""
    T = gell_mann()
    return np.real(-2j * np.einsum("aij,...ji->...a", T, G))
