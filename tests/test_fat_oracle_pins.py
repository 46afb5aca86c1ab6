"""Pins of the fat-link (asqtad / HISQ smearing) oracle against what the paper and the
mathematics fix: the path counts of the asqtad matrix, closed forms on the unit field
and on a constant abelian flux, an independent enumeration of every term, gauge
covariance, the plaquette-staple special case of the gauge oracle, and finite
differences of the smeared-link functional in complex and in group directions.
"""
import numpy as np
import pytest

import gaugegen
import oracle
from oracle import brute

# distinct, generic coefficients, so that a swapped or dropped class shows up
C_GENERIC = (0.61, -0.071, 0.013, -0.0029, -0.055, -0.043)
# tree-level asqtad values (Lepage, Phys. Rev. D 59 (1999) 074502), without tadpole factors
C_ASQTAD = (5 / 8, -1 / 16, 1 / 64, -1 / 384, -1 / 16, -1 / 24)


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _phi(U, L, c, GV, GW):
    V, W = oracle.fat_links(U, L, c)
    return float(np.real(np.sum(np.conj(GV) * V) + np.sum(np.conj(GW) * W)))


# --------------------------------------------------------------------- paths

def test_path_table_counts_and_shapes():
    total = 0
    for mu in range(4):
        ln, cls, d = oracle.fat_paths(mu)
        assert len(ln) == 86
        # one-link, three-, five-, seven-staple, Lepage, Naik
        np.testing.assert_array_equal(np.bincount(cls, minlength=6), [1, 6, 24, 48, 6, 1])
        np.testing.assert_array_equal(ln[cls == 0], 1)
        np.testing.assert_array_equal(ln[cls == 1], 3)
        np.testing.assert_array_equal(ln[cls == 2], 5)
        np.testing.assert_array_equal(ln[cls == 3], 7)
        np.testing.assert_array_equal(ln[cls == 4], 5)
        np.testing.assert_array_equal(ln[cls == 5], 3)
        seen = set()
        for i in range(86):
            steps = list(d[i, :ln[i]])
            assert all(s != 0 for s in steps)
            disp = np.zeros(4, dtype=int)
            for s in steps:
                disp[abs(s) - 1] += np.sign(s)
            want = np.zeros(4, dtype=int)
            want[mu] = 3 if cls[i] == 5 else 1
            np.testing.assert_array_equal(disp, want)
            # exactly one step along +mu (three for Naik), never along -mu, no backtracking
            assert steps.count(mu + 1) == (3 if cls[i] == 5 else 1)
            assert -(mu + 1) not in steps
            assert all(steps[j + 1] != -steps[j] for j in range(len(steps) - 1))
            seen.add(tuple(steps))
        assert len(seen) == 86
        # each oriented path of the fermion matrix: +mu and -mu versions of the 86
        total += 2 * 86
    # 8 + 8 + 48 + 192 + 384 + 48 = 688 (the count in the asqtad section)
    assert total == 688


# --------------------------------------------------------------- forward links

def test_unit_field():
    L = (4, 4, 4, 6)
    U = gaugegen.unit_links(L)
    V, W = oracle.fat_links(U, L, C_GENERIC)
    c1, c3, c5, c7, cL, cN = C_GENERIC
    n = c1 + 6 * c3 + 24 * c5 + 48 * c7 + 6 * cL
    np.testing.assert_allclose(V, n * U, rtol=0, atol=1e-15)
    np.testing.assert_allclose(W, cN * U, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", [1, 2])
def test_abelian_flux_closed_form(k):
    """Constant flux 2 pi k / Lx through the x-y planes (U_y = exp(i Phi x H), H = diag(1,-1,0)).

    Every path of class X picks up the phases of its y steps only: for V_x the three-staples
    give c_3 (2 cos(Phi H) + 4), five-staples c_5 (16 cos(Phi H) + 8), seven-staples
    48 c_7 cos(Phi H), Lepage c_L (2 cos(2 Phi H) + 4); V_y is the same times exp(i Phi x H);
    V_z, V_t are the unit-field value; W_y = c_N exp(3 i Phi x H), the other W are c_N.
    """
    L = (6, 4, 4, 4)
    U = gaugegen.abelian_flux_links(L, k)
    V, W = oracle.fat_links(U, L, C_GENERIC)
    c1, c3, c5, c7, cL, cN = C_GENERIC
    phi = 2 * np.pi * k / L[0]
    h = np.array([1.0, -1.0, 0.0])
    C1, C2 = np.cos(phi * h), np.cos(2 * phi * h)
    D = c1 + c3 * (2 * C1 + 4) + c5 * (16 * C1 + 8) + 48 * c7 * C1 + cL * (2 * C2 + 4)
    n = c1 + 6 * c3 + 24 * c5 + 48 * c7 + 6 * cL
    x = np.arange(L[0])
    for xi in x:
        ph = np.exp(1j * phi * xi * h)
        np.testing.assert_allclose(V[:, :, :, xi, 0], np.broadcast_to(np.diag(D), V[:, :, :, xi, 0].shape),
                                   atol=1e-14)
        np.testing.assert_allclose(V[:, :, :, xi, 1], np.broadcast_to(np.diag(D * ph), V[:, :, :, xi, 1].shape),
                                   atol=1e-14)
        np.testing.assert_allclose(W[:, :, :, xi, 1],
                                   np.broadcast_to(np.diag(cN * ph ** 3), W[:, :, :, xi, 1].shape), atol=1e-14)
    eye = np.eye(3)
    np.testing.assert_allclose(V[..., 2, :, :], np.broadcast_to(n * eye, V[..., 2, :, :].shape), atol=1e-14)
    np.testing.assert_allclose(V[..., 3, :, :], np.broadcast_to(n * eye, V[..., 3, :, :].shape), atol=1e-14)
    np.testing.assert_allclose(W[..., 0, :, :], np.broadcast_to(cN * eye, W[..., 0, :, :].shape), atol=1e-15)


def test_brute_force_enumeration():
    L = (4, 4, 4, 6)
    U = gaugegen.haar_links(L, 0)
    V, W = oracle.fat_links(U, L, C_GENERIC)
    Vb, Wb = brute.fat_links(U, C_GENERIC)
    assert np.abs(V - Vb).max() <= 1e-13 * np.abs(Vb).max()
    assert np.abs(W - Wb).max() <= 1e-14


def test_gauge_covariance():
    """Every path runs from p to p+mu (Naik: p+3mu): V -> g_p V g_{p+mu}^dag, W -> g_p W g_{p+3mu}^dag."""
    L = (4, 6, 4, 4)
    U = gaugegen.haar_links(L, 2)
    g = gaugegen.gauge_transform(L, 3)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ _dag(np.roll(g, -1, axis=3 - mu))
    V, W = oracle.fat_links(U, L, C_GENERIC)
    Vg, Wg = oracle.fat_links(Ug, L, C_GENERIC)
    for mu in range(4):
        np.testing.assert_allclose(Vg[..., mu, :, :], g @ V[..., mu, :, :] @ _dag(np.roll(g, -1, axis=3 - mu)),
                                   atol=1e-13)
        np.testing.assert_allclose(Wg[..., mu, :, :], g @ W[..., mu, :, :] @ _dag(np.roll(g, -3, axis=3 - mu)),
                                   atol=1e-14)


def test_three_staple_is_plaquette_staple_of_gauge_force():
    """c = (0,1,0,0,0,0): V_{k,rho} is the sum of the 6 three-link paths k -> k+rho, the
    conjugates of the plaquette staples t_plaq of the gauge-force algorithm of Sec. II."""
    L = (4, 4, 6, 4)
    U = gaugegen.haar_links(L, 4)
    V, _ = oracle.fat_links(U, L, (0, 1, 0, 0, 0, 0))
    t = oracle.staple_sums(U, L)[..., 0, :, :]
    np.testing.assert_allclose(V, _dag(t), atol=1e-13)


# ------------------------------------------------------------------ gradient

@pytest.mark.parametrize("with_naik", [True, False])
def test_gradient_finite_differences_complex_directions(with_naik):
    """dPhi = Re sum tr(grad^dag dU) for arbitrary complex variations of all links."""
    L = (4, 4, 4, 4)
    rng = np.random.default_rng(11)
    U = gaugegen.haar_links(L, 5)
    GV = _rand_c(rng, U.shape)
    GW = _rand_c(rng, U.shape) if with_naik else np.zeros_like(U)
    grad = oracle.fat_grad(U, L, C_GENERIC, GV, GW if with_naik else None)
    for trial in range(3):
        E = _rand_c(rng, U.shape)
        eps = 1e-5
        fd = (_phi(U + eps * E, L, C_GENERIC, GV, GW) - _phi(U - eps * E, L, C_GENERIC, GV, GW)) / (2 * eps)
        an = float(np.real(np.sum(np.conj(grad) * E)))
        assert abs(fd - an) <= 1e-8 * abs(an), (trial, fd, an)


def test_force_finite_differences_group_directions():
    """dPhi/domega^a = -2i tr(T_a G) along U_{k,rho} -> exp(i eps T_a) U_{k,rho}, per link and generator."""
    L = (4, 4, 4, 6)
    rng = np.random.default_rng(12)
    U = gaugegen.near_thermal_links(L, 0.4, 6)
    GV = _rand_c(rng, U.shape)
    GW = _rand_c(rng, U.shape)
    grad = oracle.fat_grad(U, L, C_ASQTAD, GV, GW)
    G = oracle.fat_force_from_grad(U, grad)
    # G is antihermitian and traceless
    np.testing.assert_allclose(G, -_dag(G), atol=1e-14)
    assert np.abs(np.trace(G, axis1=-2, axis2=-1)).max() < 1e-14
    T = oracle.gell_mann()
    want = oracle.lie_derivative(G)
    V = L[0] * L[1] * L[2] * L[3]
    eps = 1e-4
    worst = 0.0
    for trial in range(6):
        s = int(rng.integers(V))
        mu = int(rng.integers(4))
        t, z, y, x = np.unravel_index(s, (L[3], L[2], L[1], L[0]))
        for a in range(8):
            vals = []
            for sg in (1, -1):
                Up = U.copy()
                w, v = np.linalg.eigh(sg * eps * T[a])
                Up[t, z, y, x, mu] = (v * np.exp(1j * w)) @ _dag(v) @ U[t, z, y, x, mu]
                vals.append(_phi(Up, L, C_ASQTAD, GV, GW))
            fd = (vals[0] - vals[1]) / (2 * eps)
            worst = max(worst, abs(fd - want[t, z, y, x, mu, a]) / np.abs(want).max())
    assert worst <= 1e-7, worst


@pytest.mark.parametrize("L", [(4, 4, 6, 4), (4, 4, 4, 10)])
def test_gradient_sampled_links_equal_full(L):
    """The whole field comes from the path scatter (each path instance deposits at each
    of its links), single links from the gather of the algorithm after eq. 18_7_24_7:
    the two formulations agree on every link, to rounding. Lt = 10 takes the scatter's
    parallel t-slice phases, Lt = 4 its serial order."""
    rng = np.random.default_rng(13)
    U = gaugegen.haar_links(L, 7)
    GV, GW = _rand_c(rng, U.shape), _rand_c(rng, U.shape)
    full = oracle.fat_grad(U, L, C_GENERIC, GV, GW)
    V = L[0] * L[1] * L[2] * L[3]
    sites = np.repeat(np.arange(V), 4)
    mus = np.tile(np.arange(4), V)
    part = oracle.fat_grad_links(U, L, C_GENERIC, GV, GW, sites, mus)
    flat = full.reshape(V, 4, 3, 3)
    assert np.abs(part - flat[sites, mus]).max() <= 1e-13 * np.abs(flat).max()
    assert np.abs(flat).max() > 0.1


def test_gradient_linear_in_adjoint_and_class_additive():
    L = (4, 4, 4, 4)
    rng = np.random.default_rng(14)
    U = gaugegen.haar_links(L, 8)
    G1, G2 = _rand_c(rng, U.shape), _rand_c(rng, U.shape)
    a = oracle.fat_grad(U, L, C_GENERIC, G1 + 2.5 * G2)
    b = oracle.fat_grad(U, L, C_GENERIC, G1) + 2.5 * oracle.fat_grad(U, L, C_GENERIC, G2)
    np.testing.assert_allclose(a, b, atol=1e-12)
    parts = 0
    for k in range(5):
        c = [0.0] * 6
        c[k] = C_GENERIC[k]
        parts = parts + oracle.fat_grad(U, L, c, G1)
    np.testing.assert_allclose(parts, oracle.fat_grad(U, L, C_GENERIC, G1), atol=1e-12)


def test_sampled_links_equal_full():
    L = (4, 6, 4, 4)
    rng = np.random.default_rng(16)
    U = gaugegen.haar_links(L, 10)
    V, W = oracle.fat_links(U, L, C_GENERIC)
    n = L[0] * L[1] * L[2] * L[3]
    sites = rng.integers(0, n, 30)
    mus = rng.integers(0, 4, 30)
    Vs, Ws = oracle.fat_links_links(U, L, C_GENERIC, sites, mus)
    np.testing.assert_array_equal(Vs, V.reshape(n, 4, 3, 3)[sites, mus])
    np.testing.assert_array_equal(Ws, W.reshape(n, 4, 3, 3)[sites, mus])
