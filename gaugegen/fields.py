"""Seeded field generators (recipes G1-G4 and closed-form test fields)."""
import numpy as np

_CHUNK = 1 << 20  # matrices per eigh call; keeps temporaries bounded on large lattices


def field_shape(L, extra=(4, 3, 3)):
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return (Lt, Lz, Ly, Lx) + tuple(extra)


def generators():
    """Gell-Mann matrices / 2: Hermitian, traceless, tr(T_a T_b) = delta_ab / 2."""
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


def haar_su3(rng, shape):
    """G1: Haar-random SU(3) matrices of the given batch shape.

    Z = (N(0,1) + i N(0,1))/sqrt(2) (real block drawn first, then imaginary);
    Q, R = qr(Z); Q <- Q diag(R_ii/|R_ii|) (Haar on U(3), Mezzadri 2007);
    U = Q det(Q)^(-1/3) with the principal cube root.
    """
    shape = tuple(shape)
    re = rng.standard_normal(shape + (3, 3))
    im = rng.standard_normal(shape + (3, 3))
    Z = (re + 1j * im) / np.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(Q)
    return Q * (det ** (-1.0 / 3.0))[..., None, None]


def haar_links(L, seed):
    """Config recipe G1: every link Haar-random (seeded)."""
    rng = np.random.default_rng(seed)
    return haar_su3(rng, field_shape(L, (4,)))


def _exp_i_hermitian(H):
    """exp(iH) for a stack of Hermitian matrices via the spectral decomposition."""
    out = np.empty_like(H)
    flat_in = H.reshape(-1, 3, 3)
    flat_out = out.reshape(-1, 3, 3)
    for a in range(0, flat_in.shape[0], _CHUNK):
        w, v = np.linalg.eigh(flat_in[a:a + _CHUNK])
        flat_out[a:a + _CHUNK] = (v * np.exp(1j * w)[:, None, :]) @ np.conj(np.swapaxes(v, -1, -2))
    return out


def near_thermal_links(L, eps, seed):
    """Config recipe G2: U = exp(i eps sum_a r_a T_a), r_a ~ N(0,1) of shape (..., 4, 8)."""
    rng = np.random.default_rng(seed)
    r = rng.standard_normal(field_shape(L, (4, 8)))
    H = eps * np.einsum("...a,aij->...ij", r, generators())
    return _exp_i_hermitian(H)


def near_thermal_links_device(L, eps, seed, device, dtype=None):
    """Recipe G2 with the same seeded normals, exponentiated on `device` with
    torch.linalg.matrix_exp in complex128 (for large benchmark batches). Equal to
    near_thermal_links up to rounding; returns a complex128 torch tensor (or dtype)."""
    import torch

    rng = np.random.default_rng(seed)
    r = torch.from_numpy(rng.standard_normal(field_shape(L, (4, 8)))).to(device)
    T = torch.from_numpy(generators()).to(device)
    H = eps * torch.einsum("...a,aij->...ij", r.to(T.dtype), T)
    U = torch.linalg.matrix_exp(1j * H)
    return U if dtype is None else U.to(dtype)


def momenta(L, seed):
    """Config recipe G3: Pi = i sum_a p_a T_a with p_a ~ N(0,1) of shape (..., 4, 8).

    Pi is antihermitian and traceless; the kinetic energy -tr(Pi^2) = sum_a p_a^2 / 2.
    """
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(field_shape(L, (4, 8)))
    return 1j * np.einsum("...a,aij->...ij", p, generators())


def gauge_transform(L, seed):
    """Recipe G4: one Haar SU(3) matrix per site, shape (Lt, Lz, Ly, Lx, 3, 3)."""
    rng = np.random.default_rng(seed)
    return haar_su3(rng, field_shape(L, ()))


def unit_links(L):
    """Every link the identity."""
    U = np.zeros(field_shape(L), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def abelian_flux_links(L, k=1):
    """Constant abelian flux through the x-y planes.

    U_{n,y} = exp(i Phi x_n H) with H = diag(1, -1, 0), Phi = 2 pi k / Lx; every other
    link is the identity. Periodic in x because Phi Lx is a multiple of 2 pi.
    """
    Lx = int(L[0])
    U = unit_links(L)
    phi = 2.0 * np.pi * k / Lx
    x = np.arange(Lx)
    diag = np.stack([np.exp(1j * phi * x), np.exp(-1j * phi * x), np.ones(Lx)], axis=-1)
    Uy = np.zeros((Lx, 3, 3), dtype=np.complex128)
    Uy[:, 0, 0], Uy[:, 1, 1], Uy[:, 2, 2] = diag[:, 0], diag[:, 1], diag[:, 2]
    U[:, :, :, :, 1] = Uy[None, None, None, :]
    return U


# The five workloads: lattice, link recipe and seeds. u0 = 0.8677 and beta = 3.0 throughout.
CONFIGS = {
    "haar_4x4x4x4": dict(L=(4, 4, 4, 4), recipe="haar", seed=0),
    "thermal_16x16x16x32": dict(L=(16, 16, 16, 32), recipe="thermal", eps=0.3, seed=1),
    "thermal_32x32x32x64": dict(L=(32, 32, 32, 64), recipe="thermal", eps=0.25, seed=2),
    "thermal_24x24x24x48": dict(L=(24, 24, 24, 48), recipe="thermal", eps=0.3, seed=3,
                                momenta_seed=4, fd_seed=5),
}
U0 = 0.8677
BETA = 3.0


def make_config(name):
    """Link field of a named workload."""
    cfg = CONFIGS[name]
    if cfg["recipe"] == "haar":
        return haar_links(cfg["L"], cfg["seed"])
    return near_thermal_links(cfg["L"], cfg["eps"], cfg["seed"])


def batch_recipe(n=64, master_seed=6):
    """Config 5 recipe: n lattices with sizes uniform over {8^4, 12^4, 16^3x32} and
    eps ~ U[0.2, 0.4], each with its own child seed of SeedSequence(master_seed)."""
    children = np.random.SeedSequence(master_seed).spawn(n)
    sizes = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32)]
    out = []
    for ch in children:
        rng = np.random.default_rng(ch)
        L = sizes[int(rng.integers(0, 3))]
        eps = float(rng.uniform(0.2, 0.4))
        seed = int(rng.integers(0, 2**31 - 1))
        out.append(dict(L=L, eps=eps, seed=seed))
    return out
