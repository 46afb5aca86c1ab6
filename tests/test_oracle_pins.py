"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms, exact
symmetries, an independent brute-force enumeration, a textbook routine, finite
differences of the action, or invariants of the integrator. A plausible mistake in
the oracle (a dropped loop, a wrong sign, a transposed operand, a wrong neighbour)
fails at least one of them.
"""
import numpy as np
import pytest

import gaugegen
import oracle
from oracle import brute

U0, BETA = 0.8677, 3.0


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


# ------------------------------------------------------------------ coefficients

def test_coeffs_special_values():
    # u0 = 1: alpha_s = 0, so c_rect = -1/20 and c_cube = 0 exactly.
    c, a = oracle.coeffs(1.0)
    assert a == 0.0
    np.testing.assert_allclose(c, [1.0, -0.05, 0.0], rtol=0, atol=1e-16)
    # the alpha_s formula uses the natural log: u0 = exp(-3.06839/4) gives alpha_s = 1,
    # then c_rect = -(1 + 0.4805)/(20 u0^2), c_cube = -2 * 0.03325 / u0^2.
    u0 = np.exp(-3.06839 / 4)
    c, a = oracle.coeffs(u0)
    assert abs(a - 1.0) < 1e-14
    assert abs(c[1] * 20 * u0 * u0 + 1.4805) < 1e-13
    assert abs(c[2] * u0 * u0 + 0.0665) < 1e-15
    # u0 < 1 makes alpha_s positive and both improvement terms negative
    c, a = oracle.coeffs(U0)
    assert a > 0 and c[1] < -0.05 and c[2] < 0
    with pytest.raises(ValueError):
        oracle.coeffs(0.0)


# ---------------------------------------------------------------------- loop set

def test_loop_table_counts_and_closure():
    ln, cl, d = oracle.loop_table()
    assert len(ln) == 34
    assert [int((cl == k).sum()) for k in range(3)] == [6, 12, 16]
    for i in range(34):
        steps = d[i, : ln[i]]
        disp = np.zeros(4, int)
        visited = set()
        pos = np.zeros(4, int)
        for s in steps:
            a = abs(s) - 1
            nxt = pos.copy()
            nxt[a] += 1 if s > 0 else -1
            edge = (tuple(np.minimum(pos, nxt)), a)
            assert edge not in visited, "a loop must not reuse a link"
            visited.add(edge)
            pos = nxt
            disp[a] += 1 if s > 0 else -1
        assert not disp.any(), "every loop closes"
    # staples per link direction: 6 plaquette, 18 rectangle, 24 cube (48 in all)
    for rho in range(1, 5):
        per = [0, 0, 0]
        for i in range(34):
            per[cl[i]] += int(np.sum(np.abs(d[i, : ln[i]]) == rho))
        assert per == [6, 18, 24]


# ---------------------------------------------------------------- closed forms

def test_unit_field(coeffs):
    L = (4, 4, 4, 6)
    V = 4 * 4 * 4 * 6
    U = gaugegen.unit_links(L)
    S, W = oracle.action(U, L, coeffs, BETA)
    assert S == 0.0
    np.testing.assert_array_equal(W / V, [18.0, 36.0, 48.0])
    # the loop sum per site on the unit field is 3 * sum over the 34 loops of c_P
    assert abs(np.dot(W / V, coeffs) - 3 * (6 + 12 * coeffs[1] + 16 * coeffs[2])) < 1e-12
    assert np.abs(oracle.force(U, L, coeffs, BETA)).max() == 0.0


def _abelian_closed_form(L, k, c, beta):
    V = np.prod(L)
    phi = 2 * np.pi * k / L[0]
    return beta / 3 * V * (2 * (1 - np.cos(phi)) * (1 + 8 * c[2]) + 4 * c[1] * (1 - np.cos(2 * phi)))


@pytest.mark.parametrize("L,k", [((4, 4, 4, 4), 1), ((6, 4, 4, 4), 1), ((8, 4, 6, 4), 3)])
def test_abelian_flux_closed_form(coeffs, L, k):
    """Constant abelian flux in the x-y planes: plaquettes see Phi, x-y rectangles 2 Phi,
    the 8 cube loops per site spanning x and y see Phi; all other loops are trivial."""
    U = gaugegen.abelian_flux_links(L, k)
    S, _ = oracle.action(U, L, coeffs, BETA)
    expect = _abelian_closed_form(L, k, coeffs, BETA)
    assert abs(S - expect) <= 1e-12 * abs(expect)
    # a constant field strength is a stationary point: the force vanishes
    assert np.abs(oracle.force(U, L, coeffs, BETA)).max() < 1e-14


def test_abelian_value_4444():
    c, _ = oracle.coeffs(U0)
    S, _ = oracle.action(gaugegen.abelian_flux_links((4, 4, 4, 4), 1), (4, 4, 4, 4), c, BETA)
    assert abs(S - 296.9763113914771) < 1e-10


def test_abelian_detects_a_dropped_cube_term(coeffs):
    """Sensitivity of the closed form: the same field with the cube term removed is off."""
    L = (4, 4, 4, 4)
    U = gaugegen.abelian_flux_links(L, 1)
    wrong = coeffs.copy()
    wrong[2] = 0.0
    S, _ = oracle.action(U, L, wrong, BETA)
    assert abs(S - _abelian_closed_form(L, 1, coeffs, BETA)) > 1.0


# ----------------------------------------------------- independent enumerations

@pytest.mark.parametrize("L,seed", [((4, 4, 4, 4), 0), ((4, 6, 4, 4), 11)])
def test_brute_force_enumeration(coeffs, L, seed):
    U = gaugegen.haar_links(L, seed)
    S, W = oracle.action(U, L, coeffs, BETA)
    Sb, Wb = brute.action(U, coeffs, BETA)
    np.testing.assert_allclose(W, Wb, rtol=1e-13, atol=1e-10)
    assert abs(S - Sb) <= 1e-13 * abs(S)


def test_wilson_special_case():
    """c = (1, 0, 0) reduces S_G to the textbook Wilson plaquette action."""
    L = (4, 4, 6, 4)
    U = gaugegen.haar_links(L, 3)
    S, _ = oracle.action(U, L, [1.0, 0.0, 0.0], BETA)
    Sw = brute.wilson_action(U, BETA)
    assert abs(S - Sw) <= 1e-13 * abs(Sw)


# --------------------------------------------------------------------- symmetries

def _gauge(U, g):
    Ug = np.empty_like(U)
    for mu in range(4):
        g_fwd = np.roll(g, -1, axis=3 - mu)
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ _dag(g_fwd)
    return Ug


def test_gauge_invariance_and_covariance(coeffs):
    L = (4, 4, 4, 4)
    U = gaugegen.haar_links(L, 0)
    g = gaugegen.gauge_transform(L, 21)
    Ug = _gauge(U, g)
    S, _ = oracle.action(U, L, coeffs, BETA)
    Sg, _ = oracle.action(Ug, L, coeffs, BETA)
    assert abs(S - Sg) <= 1e-13 * abs(S)
    G = oracle.force(U, L, coeffs, BETA)
    Gg = oracle.force(Ug, L, coeffs, BETA)
    expect = g[..., None, :, :] @ G @ _dag(g)[..., None, :, :]
    assert np.abs(Gg - expect).max() < 1e-13 * np.abs(G).max()


def test_translation_symmetry(coeffs):
    L = (4, 6, 4, 4)
    U = gaugegen.near_thermal_links(L, 0.4, 5)
    S, _ = oracle.action(U, L, coeffs, BETA)
    G = oracle.force(U, L, coeffs, BETA)
    for axis, k in [(0, 1), (1, 2), (3, 3)]:
        Ut = np.roll(U, k, axis=3 - axis)
        St, _ = oracle.action(Ut, L, coeffs, BETA)
        assert abs(St - S) <= 1e-13 * abs(S)
        np.testing.assert_allclose(oracle.force(Ut, L, coeffs, BETA), np.roll(G, k, axis=3 - axis),
                                   rtol=0, atol=1e-13)


def test_axis_permutation_and_conjugation(coeffs):
    L = (4, 4, 4, 4)
    U = gaugegen.haar_links(L, 7)
    S, _ = oracle.action(U, L, coeffs, BETA)
    # swap lattice axes x <-> z: array axes 3 <-> 1 and directions 0 <-> 2
    Up = np.swapaxes(U, 1, 3)[..., [2, 1, 0, 3], :, :]
    Sp, _ = oracle.action(np.ascontiguousarray(Up), L, coeffs, BETA)
    assert abs(Sp - S) <= 1e-13 * abs(S)
    # cyclic permutation x->y->z->t->x
    Uc = np.transpose(U, (1, 2, 3, 0, 4, 5, 6))[..., [3, 0, 1, 2], :, :]
    Sc, _ = oracle.action(np.ascontiguousarray(Uc), L, coeffs, BETA)
    assert abs(Sc - S) <= 1e-13 * abs(S)
    # complex conjugation leaves Re tr of every loop unchanged
    Sk, _ = oracle.action(np.conj(U), L, coeffs, BETA)
    assert abs(Sk - S) <= 1e-13 * abs(S)


# ------------------------------------------------------------- force structure

def test_force_is_traceless_antihermitian(coeffs):
    L = (4, 4, 4, 4)
    G = oracle.force(gaugegen.haar_links(L, 0), L, coeffs, BETA)
    assert np.abs(G + _dag(G)).max() < 1e-15
    assert np.abs(np.trace(G, axis1=-2, axis2=-1)).max() < 1e-15


def test_staple_sum_action_identity(coeffs):
    """sum over links of Re tr(U t^X) = L_X W_X: every loop of class X is seen once from
    each of its L_X links (4 for plaquettes, 6 for rectangles and cubes)."""
    L = (4, 4, 6, 4)
    U = gaugegen.near_thermal_links(L, 0.5, 9)
    t = oracle.staple_sums(U, L)
    _, W = oracle.action(U, L, coeffs, BETA)
    lhs = np.einsum("tzyxmij,tzyxmcji->c", U, t).real
    np.testing.assert_allclose(lhs, np.array([4, 6, 6]) * W, rtol=1e-13)


# ------------------------------------------------------------ finite differences

def _fd(U, L, c, site, mu, a, eps, local):
    T = oracle.gell_mann()
    idx = np.unravel_index(site, U.shape[:4])
    vals = []
    for sg in (1, -1):
        U2 = U.copy()
        U2[idx + (mu,)] = oracle.su3_exp(1j * sg * eps * T[a]) @ U2[idx + (mu,)]
        if local:
            vals.append(oracle.local_action(U2, L, c, BETA, site, mu))
        else:
            vals.append(oracle.action(U2, L, c, BETA)[0])
    return (vals[0] - vals[1]) / (2 * eps)


def test_force_matches_finite_differences_full_action(coeffs):
    """dS/domega^a = -2i tr(T_a G) along U -> exp(i eps T_a) U, central differences."""
    L = (4, 4, 4, 4)
    U = gaugegen.haar_links(L, 0)
    G = oracle.force(U, L, coeffs, BETA)
    d = oracle.lie_derivative(G)
    rng = np.random.default_rng(1)
    for _ in range(6):
        site, mu, a = int(rng.integers(256)), int(rng.integers(4)), int(rng.integers(8))
        idx = np.unravel_index(site, U.shape[:4])
        fd = _fd(U, L, coeffs, site, mu, a, 1e-4, local=False)
        assert abs(fd - d[idx + (mu, a)]) <= 1e-6 * max(1.0, abs(d[idx + (mu, a)]))


def test_force_matches_finite_differences_local_action():
    """Same on a larger, near-thermal lattice with the local action of the link, and with
    the Wilson coefficients (plaquette-only force)."""
    L = (8, 6, 6, 8)
    U = gaugegen.near_thermal_links(L, 0.3, 5)
    rng = np.random.default_rng(2)
    for c in (oracle.coeffs(U0)[0], np.array([1.0, 0.0, 0.0])):
        sites = rng.integers(0, np.prod(L), 5)
        mus = rng.integers(0, 4, 5)
        G = oracle.force_links(U, L, c, BETA, sites, mus)
        d = oracle.lie_derivative(G)
        for i in range(5):
            for a in (0, 3, 7):
                fd = _fd(U, L, c, int(sites[i]), int(mus[i]), a, 1e-4, local=True)
                assert abs(fd - d[i, a]) <= 1e-6 * max(1.0, np.abs(d[i]).max())


def test_local_action_carries_the_link_dependence(coeffs):
    L = (4, 4, 4, 6)
    U = gaugegen.haar_links(L, 4)
    site, mu = 37, 2
    idx = np.unravel_index(site, U.shape[:4])
    U2 = U.copy()
    U2[idx + (mu,)] = gaugegen.haar_su3(np.random.default_rng(0), ())
    dS = oracle.action(U2, L, coeffs, BETA)[0] - oracle.action(U, L, coeffs, BETA)[0]
    dl = oracle.local_action(U2, L, coeffs, BETA, site, mu) - oracle.local_action(U, L, coeffs, BETA, site, mu)
    assert abs(dS - dl) < 1e-10


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (4, 6, 4, 6), (4, 4, 6, 8)])
def test_force_links_equals_full_force(coeffs, L):
    """The whole field comes from the loop scatter (each loop instance deposits its
    staple into every link it contains), single links from the gather by the rotation
    rules of the force algorithm: the two formulations agree on every link, to
    rounding. (4,4,6,8) takes the scatter's parallel t-slice phases, the other two its
    serial order."""
    U = gaugegen.haar_links(L, 0)
    V = int(np.prod(L))
    G = oracle.force(U, L, coeffs, BETA).reshape(V, 4, 3, 3)
    sites = np.repeat(np.arange(V), 4)
    mus = np.tile(np.arange(4), V)
    Gs = oracle.force_links(U, L, coeffs, BETA, sites, mus)
    err = np.abs(Gs - G[sites, mus]).max() / np.abs(G).max()
    assert err < 1e-13
    assert np.abs(G).max() > 0.1


def test_scatter_force_does_not_depend_on_the_thread_count(coeffs):
    """The scatter orders every link's deposits by t-slice phase, so the whole-field
    force (and the fat-link gradient) is bitwise the same on one thread and on many."""
    L = (4, 4, 4, 8)
    U = gaugegen.haar_links(L, 3)
    Lf = (4, 4, 4, 10)  # the fat paths reach two steps back and forth: phases of 5 slices
    Uf = gaugegen.haar_links(Lf, 4)
    rng = np.random.default_rng(5)
    GV = rng.standard_normal(Uf.shape) + 1j * rng.standard_normal(Uf.shape)
    GW = rng.standard_normal(Uf.shape) + 1j * rng.standard_normal(Uf.shape)
    cf = (0.61, -0.071, 0.013, -0.0029, -0.055, -0.043)
    before = oracle.set_num_threads(0)
    out = []
    try:
        for n in (1, max(2, before)):
            oracle.set_num_threads(n)
            out.append((oracle.force(U, L, coeffs, BETA), oracle.staple_sums(U, L),
                        oracle.fat_grad(Uf, Lf, cf, GV, GW)))
    finally:
        oracle.set_num_threads(before)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------- exponential map

def test_su3_exp_against_eigendecomposition():
    rng = np.random.default_rng(3)
    T = oracle.gell_mann()
    for scale in (1e-3, 0.3, 2.0, 9.0):
        w = rng.standard_normal((50, 8)) * scale
        H = np.einsum("na,aij->nij", w, T)
        X = 1j * H
        E = oracle.su3_exp(X)
        lam, v = np.linalg.eigh(H)
        ref = (v * np.exp(1j * lam)[:, None, :]) @ _dag(v)
        assert np.abs(E - ref).max() < 2e-14 * max(1.0, scale)
        eye = np.eye(3)
        assert np.abs(E @ _dag(E) - eye).max() < 1e-14 * max(1.0, scale)
        assert np.abs(np.linalg.det(E) - 1).max() < 1e-13 * max(1.0, scale)
        assert np.abs(E @ oracle.su3_exp(-X) - eye).max() < 1e-13 * max(1.0, scale)


# ------------------------------------------------------------ molecular dynamics

def test_kinetic_energy_of_generated_momenta():
    L = (4, 4, 4, 4)
    P = gaugegen.momenta(L, 4)
    T = oracle.gell_mann()
    p = np.real(-2j * np.einsum("aij,...ji->...a", T, P))  # Pi = i sum p_a T_a
    assert abs(oracle.kinetic(P, L) - 0.5 * np.sum(p * p)) < 1e-10


def test_leapfrog_unit_field_is_fixed(coeffs):
    L = (4, 4, 4, 4)
    U = gaugegen.unit_links(L)
    P = np.zeros_like(U)
    U1, P1, H0, H1 = oracle.leapfrog(U, P, L, coeffs, BETA, 0.02, 3)
    assert H0 == 0.0 and H1 == 0.0
    np.testing.assert_array_equal(U1, U)
    assert np.abs(P1).max() == 0.0


def test_leapfrog_reversibility(coeffs):
    L = (4, 4, 4, 4)
    U = gaugegen.near_thermal_links(L, 0.3, 3)
    P = gaugegen.momenta(L, 4)
    U1, P1, H0, H1 = oracle.leapfrog(U, P, L, coeffs, BETA, 0.05, 5)
    U2, P2, _, _ = oracle.leapfrog(U1, -P1, L, coeffs, BETA, 0.05, 5)
    assert np.abs(U2 - U).max() < 1e-12
    assert np.abs(P2 + P).max() < 1e-12


def test_leapfrog_energy_error_is_second_order(coeffs):
    """|dH| of a fixed-length trajectory falls by ~4 when dt halves (second order)."""
    L = (4, 4, 4, 4)
    U = gaugegen.near_thermal_links(L, 0.3, 3)
    P = gaugegen.momenta(L, 4)
    dH = []
    for n in (4, 8, 16):
        _, _, H0, H1 = oracle.leapfrog(U, P, L, coeffs, BETA, 0.4 / n, n)
        dH.append(abs(H1 - H0))
    r1, r2 = dH[0] / dH[1], dH[1] / dH[2]
    assert 3.3 < r1 < 4.7 and 3.6 < r2 < 4.4
    # unitarity is preserved by the exact exponential
    U1, _, _, _ = oracle.leapfrog(U, P, L, coeffs, BETA, 0.05, 8)
    assert np.abs(U1 @ _dag(U1) - np.eye(3)).max() < 1e-13
