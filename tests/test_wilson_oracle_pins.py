"""Pins of the Wilson-clover oracle against what the paper and the mathematics fix: the
Clifford algebra of the gamma matrices, the clover leaves (Q_{mu nu} = Q_{nu mu}^+, the
unit field, a constant abelian flux in closed form, the two equivalent normalisations
of the clover term), the free Wilson operator on plane waves, gamma_5-hermiticity,
gauge invariance and covariance, and finite differences of Psi = 2 Re Y^+ D X in
every generator direction, with and without the clover term."""
import numpy as np
import pytest

import gaugegen
import oracle

KAPPA, CSW = 0.1242, 1.37


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def _spinors(L, seed, n=2):
    rng = np.random.default_rng(seed)
    shape = (L[3], L[2], L[1], L[0], 4, 3)
    return [rng.standard_normal(shape) + 1j * rng.standard_normal(shape) for _ in range(n)]


def test_gamma_matrices():
    g = [oracle.gamma(mu) for mu in range(4)]
    eye = np.eye(4)
    for mu in range(4):
        np.testing.assert_array_equal(g[mu], _dag(g[mu]))
        for nu in range(4):
            np.testing.assert_allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2 * eye * (mu == nu), atol=0)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    np.testing.assert_allclose(g5 @ g5, eye, atol=0)
    np.testing.assert_allclose(g5, _dag(g5), atol=0)


def test_clover_leaves_structure():
    L = (4, 4, 4, 6)
    U = gaugegen.haar_links(L, 1)
    Q = oracle.clover_leaves(U, L)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                assert np.abs(Q[:, mu, nu]).max() == 0
            else:
                # Q_{n;mu nu} = Q_{n;nu mu}^+ (eq. 17_7_20_8)
                np.testing.assert_allclose(Q[:, mu, nu], _dag(Q[:, nu, mu]), atol=1e-14)
    Qu = oracle.clover_leaves(gaugegen.unit_links(L), L)
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                np.testing.assert_allclose(Qu[:, mu, nu], np.broadcast_to(4 * np.eye(3), Qu[:, mu, nu].shape))


def test_clover_abelian_flux_closed_form():
    """U_y = exp(i Phi x H): every x-y leaf is exp(i Phi H) traversed x then y, so
    Q_{xy} = 4 exp(i Phi H) at every site; all other planes give 4."""
    L = (6, 4, 4, 4)
    U = gaugegen.abelian_flux_links(L, 1)
    Q = oracle.clover_leaves(U, L)
    h = np.array([1.0, -1.0, 0.0])
    phi = 2 * np.pi / L[0]
    want = np.diag(4 * np.exp(1j * phi * h))
    np.testing.assert_allclose(Q[:, 0, 1], np.broadcast_to(want, Q[:, 0, 1].shape), atol=1e-14)
    np.testing.assert_allclose(Q[:, 1, 0], np.broadcast_to(want.conj(), Q[:, 1, 0].shape), atol=1e-14)
    np.testing.assert_allclose(Q[:, 2, 3], np.broadcast_to(4 * np.eye(3), Q[:, 2, 3].shape), atol=1e-14)


def test_clover_normalisations_agree():
    """A of eq. 18_7_17_3 with F = (Q_{mu nu} - Q_{nu mu})/8 (eq. 17_7_20_0_0), summed over
    mu < nu with c_sw/(4(m+4)), equals A of eq. 18_7_18_0: checked by applying D - D(c_sw = 0)."""
    L = (4, 4, 4, 4)
    U = gaugegen.haar_links(L, 2)
    (X,) = _spinors(L, 3, 1)
    Q = oracle.clover_leaves(U, L)
    g = [oracle.gamma(mu) for mu in range(4)]
    Xf = X.reshape(-1, 4, 3)
    AX = np.zeros_like(Xf)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            F = (Q[:, mu, nu] - Q[:, nu, mu]) / 8.0
            c = g[mu] @ g[nu] - g[nu] @ g[mu]
            AX += np.einsum("ab,nij,nbj->nai", c, F, Xf)
    kappa = KAPPA
    m4 = 1.0 / (2 * kappa)  # m + 4
    want = -CSW / (4 * m4) * AX
    got = (oracle.wilson_apply(U, X, L, kappa, CSW) - oracle.wilson_apply(U, X, L, kappa, 0.0)).reshape(-1, 4, 3)
    np.testing.assert_allclose(got, want, atol=1e-13)


def test_free_operator_on_plane_waves():
    """U = 1, X_n = exp(i p.n) chi: D X = [1 - kappa sum_mu (2 cos p_mu - 2i gamma_mu sin p_mu)] X."""
    L = (4, 6, 4, 8)
    U = gaugegen.unit_links(L)
    rng = np.random.default_rng(4)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    k = [1, 2, 3, 1]
    p = [2 * np.pi * k[a] / L[a] for a in range(4)]
    t, z, y, x = np.meshgrid(*[np.arange(L[a]) for a in (3, 2, 1, 0)], indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    X = phase[..., None, None] * chi
    M = np.eye(4, dtype=complex)
    for mu in range(4):
        M -= KAPPA * (2 * np.cos(p[mu]) * np.eye(4) - 2j * np.sin(p[mu]) * oracle.gamma(mu))
    want = phase[..., None, None] * (M @ chi)
    np.testing.assert_allclose(oracle.wilson_apply(U, X, L, KAPPA, CSW), want, atol=1e-13)


def test_gamma5_hermiticity():
    """(Y, D X) = (gamma_5 D gamma_5 Y, X) for the Wilson-clover operator."""
    L = (4, 4, 4, 4)
    U = gaugegen.haar_links(L, 5)
    X, Y = _spinors(L, 6)
    g5 = oracle.gamma(0) @ oracle.gamma(1) @ oracle.gamma(2) @ oracle.gamma(3)
    lhs = np.vdot(Y, oracle.wilson_apply(U, X, L, KAPPA, CSW))
    g5Y = np.einsum("ab,...bi->...ai", g5, Y)
    rhs = np.vdot(np.einsum("ab,...bi->...ai", g5, oracle.wilson_apply(U, g5Y, L, KAPPA, CSW)), X)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gauge_invariance_and_covariance():
    L = (4, 4, 6, 4)
    U = gaugegen.haar_links(L, 7)
    X, Y = _spinors(L, 8)
    g = gaugegen.gauge_transform(L, 9)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ _dag(np.roll(g, -1, axis=3 - mu))
    Xg = np.einsum("...ij,...aj->...ai", g, X)
    Yg = np.einsum("...ij,...aj->...ai", g, Y)
    p0 = oracle.wilson_psi(U, X, Y, L, KAPPA, CSW)
    p1 = oracle.wilson_psi(Ug, Xg, Yg, L, KAPPA, CSW)
    assert abs(p1 - p0) <= 1e-12 * abs(p0)
    G0 = oracle.wilson_force(U, X, Y, L, KAPPA, CSW)
    G1 = oracle.wilson_force(Ug, Xg, Yg, L, KAPPA, CSW)
    np.testing.assert_allclose(G1, g[..., None, :, :] @ G0 @ _dag(g)[..., None, :, :], atol=1e-12)


@pytest.mark.parametrize("csw", [0.0, CSW])
def test_force_finite_differences(csw):
    """dPsi/domega^a = -2i tr(T_a G) along U_{k,rho} -> exp(i eps T_a) U_{k,rho}."""
    L = (4, 4, 4, 6)
    U = gaugegen.near_thermal_links(L, 0.4, 10)
    X, Y = _spinors(L, 11)
    G = oracle.wilson_force(U, X, Y, L, KAPPA, csw)
    np.testing.assert_allclose(G, -_dag(G), atol=1e-13)
    assert np.abs(np.trace(G, axis1=-2, axis2=-1)).max() < 1e-13
    want = oracle.lie_derivative(G)
    T = oracle.gell_mann()
    rng = np.random.default_rng(12)
    eps = 1e-4
    worst = 0.0
    V = L[0] * L[1] * L[2] * L[3]
    for trial in range(8):
        s = int(rng.integers(V))
        mu = trial % 4
        t, z, y, x = np.unravel_index(s, (L[3], L[2], L[1], L[0]))
        for a in range(8):
            vals = []
            for sg in (1, -1):
                Up = U.copy()
                w, v = np.linalg.eigh(sg * eps * T[a])
                Up[t, z, y, x, mu] = (v * np.exp(1j * w)) @ _dag(v) @ U[t, z, y, x, mu]
                vals.append(oracle.wilson_psi(Up, X, Y, L, KAPPA, csw))
            fd = (vals[0] - vals[1]) / (2 * eps)
            worst = max(worst, abs(fd - want[t, z, y, x, mu, a]) / np.abs(want).max())
    assert worst <= 1e-7, worst


def test_clover_force_is_linear_in_csw_and_sampled_equals_full():
    L = (4, 6, 4, 4)
    U = gaugegen.haar_links(L, 13)
    X, Y = _spinors(L, 14)
    G0 = oracle.wilson_force(U, X, Y, L, KAPPA, 0.0)
    G1 = oracle.wilson_force(U, X, Y, L, KAPPA, 1.0)
    G2 = oracle.wilson_force(U, X, Y, L, KAPPA, 2.5)
    np.testing.assert_allclose(G2 - G0, 2.5 * (G1 - G0), atol=1e-12)
    V = L[0] * L[1] * L[2] * L[3]
    rng = np.random.default_rng(15)
    sites, mus = rng.integers(0, V, 30), rng.integers(0, 4, 30)
    part = oracle.wilson_force_links(U, X, Y, L, KAPPA, 2.5, sites, mus)
    np.testing.assert_array_equal(part, G2.reshape(V, 4, 3, 3)[sites, mus])
