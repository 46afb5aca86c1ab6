"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: FP64 force and action 1e-12 relative, FP32 force and action 1e-5 relative
(force: max over links of the Frobenius error / max over links of the reference
norm). The FP32 gate compares against the oracle evaluated on the same FP32-rounded
links promoted exactly to FP64; the end-to-end error against the unrounded links is
printed beside it.
"""
import numpy as np
import pytest
import torch

import gaugegen
import oracle
from oracle import brute

from gpu_util import device, force_errors, from_soa, rounded, soa_reference, to_soa

pytestmark = pytest.mark.gpu

U0, BETA = gaugegen.U0, gaugegen.BETA
TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def sym():
    import paper_1808_02281_amd as m

    device()
    yield m
    m.set_force_algorithm("auto")
    m.set_coeffs_override(None)


@pytest.fixture(scope="module")
def c():
    return oracle.coeffs(U0)[0]


# ------------------------------------------------------------------ layout

@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_pack_layout_and_roundtrip(sym, prec):
    L = (4, 6, 4, 8)
    U = gaugegen.haar_links(L, 5)
    dev = device()
    S = to_soa(sym, U, L, prec, dev)
    ref = soa_reference(rounded(U, prec), L)
    np.testing.assert_array_equal(S.cpu().numpy().astype(np.float64), ref)
    back = sym.unpack(S, L)
    aos = torch.from_numpy(U).to(torch.complex128 if prec == "f64" else torch.complex64).to(dev)
    assert torch.equal(back, aos)


# ------------------------------------------------------------ small lattices

SMALL = [
    ("haar_4x4x4x4", (4, 4, 4, 4), None),           # config 1; one partial tile
    ("thermal_6x6x6x8", (6, 6, 6, 8), 0.4),        # 3 full tiles and a ragged tail per block
    ("thermal_4x8x6x10", (4, 8, 6, 10), 0.5),      # non-cubic
]


def _field(name, L, eps):
    return gaugegen.haar_links(L, 0) if eps is None else gaugegen.near_thermal_links(L, eps, 17)


@pytest.mark.parametrize("alg", ["direct", "factored"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,L,eps", SMALL)
def test_force_and_action_parity_small(sym, c, alg, prec, name, L, eps):
    print(f"case {name} {prec} {alg}", flush=True)
    sym.set_force_algorithm(alg)
    U = _field(name, L, eps)
    Ur = rounded(U, prec)
    G_ref = oracle.force(Ur, L, c, BETA)
    S_ref, W_ref = oracle.action(Ur, L, c, BETA)
    dev = device()
    Us = to_soa(sym, U, L, prec, dev)
    F, S = sym.force(Us, L, U0, BETA, with_action=True)
    Sa = sym.action(Us, L, U0, BETA)
    G = from_soa(sym, F, L)
    gmax, rms, worst = force_errors(G, G_ref)
    S = S.cpu().numpy()
    Sa = Sa.cpu().numpy()
    print(f"  force gmax {gmax:.2e} rms {rms:.2e} worst-link {worst:.2e}; "
          f"S(force) {abs(S[0] - S_ref) / abs(S_ref):.2e} S(action) {abs(Sa[0] - S_ref) / abs(S_ref):.2e}")
    tol = TOL[prec]
    assert gmax <= tol
    assert abs(S[0] - S_ref) <= tol * abs(S_ref)
    assert abs(Sa[0] - S_ref) <= tol * abs(S_ref)
    np.testing.assert_allclose(Sa[1:], W_ref, rtol=tol)
    np.testing.assert_allclose(S[1:], W_ref, rtol=tol)
    if prec == "f32":
        e2e = force_errors(G, oracle.force(U, L, c, BETA))[0]
        print(f"  end-to-end FP32 force error vs unrounded links: {e2e:.2e}")


@pytest.mark.parametrize("alg", ["direct", "factored"])
def test_unit_and_abelian_fields(sym, c, alg):
    sym.set_force_algorithm(alg)
    dev = device()
    L = (4, 4, 4, 4)
    Us = to_soa(sym, gaugegen.unit_links(L), L, "f64", dev)
    F, S = sym.force(Us, L, U0, BETA, with_action=True)
    assert torch.count_nonzero(F).item() == 0
    # the action kernel sums (3 - Re tr P) = 0 exactly; the fused force action of the
    # factored path recovers the cube part as a difference of traces, exact to rounding
    assert abs(S[0].item()) <= 1e-12 * BETA * np.prod(L)
    assert sym.action(Us, L, U0, BETA)[0].item() == 0.0
    L = (8, 4, 6, 4)
    U = gaugegen.abelian_flux_links(L, 3)
    phi = 2 * np.pi * 3 / L[0]
    expect = BETA / 3 * np.prod(L) * (2 * (1 - np.cos(phi)) * (1 + 8 * c[2]) + 4 * c[1] * (1 - np.cos(2 * phi)))
    Us = to_soa(sym, U, L, "f64", dev)
    F, S = sym.force(Us, L, U0, BETA, with_action=True)
    assert abs(S[0].item() - expect) <= 1e-12 * expect
    assert abs(sym.action(Us, L, U0, BETA)[0].item() - expect) <= 1e-12 * expect
    assert torch.abs(F).max().item() < 1e-13


@pytest.mark.parametrize("alg", ["direct", "factored"])
def test_wilson_override(sym, alg):
    """c = (1, 0, 0): the action is the textbook Wilson plaquette action."""
    sym.set_force_algorithm(alg)
    L = (4, 4, 6, 4)
    U = gaugegen.haar_links(L, 3)
    dev = device()
    try:
        sym.set_coeffs_override((1.0, 0.0, 0.0))
        Us = to_soa(sym, U, L, "f64", dev)
        F, S = sym.force(Us, L, U0, BETA, with_action=True)
        Sa = sym.action(Us, L, U0, BETA)
    finally:
        sym.set_coeffs_override(None)
    Sw = brute.wilson_action(U, BETA)
    assert abs(S[0].item() - Sw) <= 1e-12 * abs(Sw)
    assert abs(Sa[0].item() - Sw) <= 1e-12 * abs(Sw)
    G_ref = oracle.force(U, L, [1.0, 0.0, 0.0], BETA)
    assert force_errors(from_soa(sym, F, L), G_ref)[0] <= 1e-12


def test_gauge_covariance_on_gpu(sym, c):
    L = (4, 6, 4, 4)
    U = gaugegen.near_thermal_links(L, 0.6, 2)
    g = gaugegen.gauge_transform(L, 8)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(np.roll(g, -1, axis=3 - mu), -1, -2))
    dev = device()
    F1, S1 = sym.force(to_soa(sym, U, L, "f64", dev), L, U0, BETA, with_action=True)
    F2, S2 = sym.force(to_soa(sym, Ug, L, "f64", dev), L, U0, BETA, with_action=True)
    G1, G2 = from_soa(sym, F1, L), from_soa(sym, F2, L)
    expect = g[..., None, :, :] @ G1 @ np.conj(np.swapaxes(g, -1, -2))[..., None, :, :]
    assert np.abs(G2 - expect).max() <= 1e-13 * np.abs(G1).max()
    assert abs(S1[0].item() - S2[0].item()) <= 1e-13 * abs(S1[0].item())


def test_action_is_deterministic(sym):
    L = (8, 8, 8, 8)
    Us = to_soa(sym, gaugegen.near_thermal_links(L, 0.3, 4), L, "f64", device())
    a = [sym.action(Us, L, U0, BETA).cpu().numpy() for _ in range(2)]
    b = [sym.force(Us, L, U0, BETA, with_action=True)[1].cpu().numpy() for _ in range(2)]
    assert np.array_equal(a[0], a[1]) and np.array_equal(b[0], b[1])


def test_error_codes_surface(sym):
    from paper_1808_02281_amd import _lib

    L = (4, 4, 4, 4)
    Us = to_soa(sym, gaugegen.unit_links(L), L, "f64", device())
    with pytest.raises(ValueError):
        sym.force(Us, (4, 4, 4, 6), U0, BETA)
    with pytest.raises(_lib.SymError) as e:
        sym.force(Us, L, -1.0, BETA)
    assert e.value.status == -1


# ------------------------------------------------------- 16^3 x 32 (config 2)

@pytest.mark.parametrize("alg", ["direct", "factored"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_parity_16x16x16x32(sym, c, alg, prec):
    print(f"case thermal_16x16x16x32 {prec} {alg}", flush=True)
    sym.set_force_algorithm(alg)
    cfg = gaugegen.CONFIGS["thermal_16x16x16x32"]
    L = cfg["L"]
    U = gaugegen.near_thermal_links(L, cfg["eps"], cfg["seed"])
    Ur = rounded(U, prec)
    G_ref = oracle.force(Ur, L, c, BETA)
    S_ref, W_ref = oracle.action(Ur, L, c, BETA)
    Us = to_soa(sym, U, L, prec, device())
    F, S = sym.force(Us, L, U0, BETA, with_action=True)
    Sa = sym.action(Us, L, U0, BETA)
    G = from_soa(sym, F, L)
    gmax, rms, worst = force_errors(G, G_ref)
    S, Sa = S.cpu().numpy(), Sa.cpu().numpy()
    print(f"  force gmax {gmax:.2e} rms {rms:.2e} worst {worst:.2e}; action(force) {abs(S[0]-S_ref)/S_ref:.2e} "
          f"action {abs(Sa[0]-S_ref)/S_ref:.2e}", flush=True)
    assert gmax <= TOL[prec]
    assert abs(S[0] - S_ref) <= TOL[prec] * abs(S_ref)
    assert abs(Sa[0] - S_ref) <= TOL[prec] * abs(S_ref)


# --------------------------------------------- 32^3 x 64 (config 3), every link

@pytest.fixture(scope="module")
def big_field():
    cfg = gaugegen.CONFIGS["thermal_32x32x32x64"]
    return cfg["L"], gaugegen.near_thermal_links(cfg["L"], cfg["eps"], cfg["seed"])


@pytest.fixture(scope="module")
def big_oracle(c, big_field):
    """The oracle's force and action on the unrounded FP64 links (every link)."""
    L, U = big_field
    return oracle.force(U, L, c, BETA), oracle.action(U, L, c, BETA)[0]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_parity_32x32x32x64_every_link(sym, c, big_field, big_oracle, prec):
    """The benchmark workload in the launch configuration the benchmark times (auto
    algorithm), compared with the oracle on all 8,388,608 links and on the action.
    FP32 is gated against the oracle on the same FP32-rounded links and, end to end,
    against the oracle on the unrounded links, both at 1e-5."""
    print(f"case thermal_32x32x32x64 {prec} every link", flush=True)
    sym.set_force_algorithm("auto")
    L, U = big_field
    G_u, S_u = big_oracle
    dev = device()
    Us = to_soa(sym, U, L, prec, dev)
    F, S = sym.force(Us, L, U0, BETA, with_action=True)
    G = from_soa(sym, F, L)
    del F, Us
    if prec == "f64":
        G_ref, S_ref = G_u, S_u
    else:
        Ur = rounded(U, prec)
        G_ref, S_ref = oracle.force(Ur, L, c, BETA), oracle.action(Ur, L, c, BETA)[0]
        del Ur
    gmax, rms, worst = force_errors(G, G_ref)
    serr = abs(S[0].item() - S_ref) / abs(S_ref)
    print(f"  every link: force max {gmax:.2e} rms {rms:.2e} worst-link {worst:.2e}; action {serr:.2e}", flush=True)
    assert gmax <= TOL[prec]
    assert serr <= TOL[prec]
    # structure of every link: antihermitian and traceless to rounding
    scale = np.abs(G).max()
    eps = np.finfo(np.float32 if prec == "f32" else np.float64).eps
    assert np.abs(G + np.conj(np.swapaxes(G, -1, -2))).max() <= 8 * eps * scale
    assert np.abs(np.trace(G, axis1=-2, axis2=-1)).max() <= 16 * eps * scale
    if prec == "f32":
        e2e = force_errors(G, G_u)
        se2e = abs(S[0].item() - S_u) / abs(S_u)
        print(f"  end to end (unrounded links): force max {e2e[0]:.2e} rms {e2e[1]:.2e}; action {se2e:.2e}",
              flush=True)
        assert e2e[0] <= TOL[prec]
        assert se2e <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_force_bitwise_repeatable_32x32x32x64(sym, big_field, prec):
    """Twenty force calls with the fused action on the benchmark workload give bitwise the
    same forces and action as the first: nothing in the passes depends on timing (each
    thread writes only its own staples and force, the reductions have a fixed order)."""
    print(f"case thermal_32x32x32x64 {prec} repeatability", flush=True)
    sym.set_force_algorithm("auto")
    L, U = big_field
    Us = to_soa(sym, U, L, prec, device())
    F0, S0 = sym.force(Us, L, U0, BETA, with_action=True)
    F = torch.empty_like(F0)
    for _ in range(20):
        _, S = sym.force(Us, L, U0, BETA, with_action=True, out=F)
        assert torch.equal(F, F0)
        assert torch.equal(S, S0)


# ------------------------------------------- fused action with c_cube = 0

@pytest.mark.parametrize("alg", ["direct", "factored"])
def test_fused_action_with_zero_cube_coefficient(sym, alg):
    """u0 = 1 gives alpha_s = 0, hence c_cube = 0: the factored partials cannot separate
    W_C, and the action kernel supplies S and W. Every output is finite and equals the
    oracle's (single lattice and batch)."""
    sym.set_force_algorithm(alg)
    L = (4, 6, 4, 8)
    U = gaugegen.near_thermal_links(L, 0.4, 31)
    c1, _ = oracle.coeffs(1.0)
    assert c1[2] == 0.0
    S_ref, W_ref = oracle.action(U, L, c1, BETA)
    G_ref = oracle.force(U, L, c1, BETA)
    dev = device()
    Us = to_soa(sym, U, L, "f64", dev)
    F, S = sym.force(Us, L, 1.0, BETA, with_action=True)
    S = S.cpu().numpy()
    assert np.isfinite(S).all()
    assert abs(S[0] - S_ref) <= 1e-12 * abs(S_ref)
    np.testing.assert_allclose(S[1:], W_ref, rtol=1e-12)
    assert force_errors(from_soa(sym, F, L), G_ref)[0] <= 1e-12
    gr, Sg = sym.action_grad(Us, L, 1.0, BETA, with_action=True)
    np.testing.assert_allclose(Sg.cpu().numpy(), S, rtol=1e-12)
    Fs, Sb = sym.force_batch([Us, Us], [L, L], 1.0, BETA, with_action=True)
    Sb = Sb.cpu().numpy()
    assert np.isfinite(Sb).all()
    for k in range(2):
        np.testing.assert_allclose(Sb[k], S, rtol=1e-12)
    sym.set_force_algorithm("auto")


# ------------------------------------------------------------- link check

def test_check_links(sym):
    """sym_check_links: max unitarity defect, max |det - 1| and the count of non-finite
    links, on fields whose answers are known."""
    L = (4, 4, 4, 6)
    dev = device()
    out = sym.check_links(to_soa(sym, gaugegen.unit_links(L), L, "f64", dev), L).cpu().numpy()
    assert out.tolist() == [0.0, 0.0, 0.0]
    U = gaugegen.haar_links(L, 12)
    out = sym.check_links(to_soa(sym, U, L, "f64", dev), L).cpu().numpy()
    assert out[0] <= 1e-14 and out[1] <= 1e-14 and out[2] == 0
    out = sym.check_links(to_soa(sym, U, L, "f32", dev), L).cpu().numpy()
    assert 1e-9 < out[0] <= 2e-6 and out[1] <= 2e-6 and out[2] == 0
    V = U.copy()
    V[1, 2, 3, 0, 2] *= 1.01           # ||U^+U - 1||_F = (1.01^2 - 1) sqrt(3), det - 1 = 1.01^3 - 1
    V[3, 0, 1, 2, 1, 0, 2] = np.nan
    V[0, 0, 0, 1, 3, 2, 2] = np.inf
    out = sym.check_links(to_soa(sym, V, L, "f64", dev), L).cpu().numpy()
    assert abs(out[0] - (1.01 ** 2 - 1) * np.sqrt(3)) <= 1e-12
    assert abs(out[1] - (1.01 ** 3 - 1)) <= 1e-12
    assert out[2] == 2


def _project_rows(M):
    """SU(3) projection by rows (numpy, double): row 0 normalised, row 1 orthogonalised
    against it and normalised, row 2 = conj(row 0 x row 1)."""
    r0 = M[..., 0, :] / np.linalg.norm(M[..., 0, :], axis=-1, keepdims=True)
    r1 = M[..., 1, :] - np.sum(np.conj(r0) * M[..., 1, :], axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    return np.stack([r0, r1, np.conj(np.cross(r0, r1))], axis=-2)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_reunitarise(sym, prec):
    """sym_reunitarise against the projection written out in numpy, on links pulled off
    SU(3) by complex noise; SU(3) links barely move; the result passes sym_check_links;
    a link with a non-finite element stays non-finite and is counted."""
    L = (4, 6, 4, 6)
    dev = device()
    rng = np.random.default_rng(17)
    U = gaugegen.haar_links(L, 13)
    V = U + 0.05 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    V = rounded(V, prec)
    want = _project_rows(V)
    Vs = to_soa(sym, V, L, prec, dev)
    got = from_soa(sym, sym.reunitarise(Vs, L), L)
    tol = 1e-14 if prec == "f64" else 4e-7
    assert np.abs(got - want).max() <= tol
    chk = sym.check_links(Vs, L).cpu().numpy()
    assert chk[0] <= (1e-14 if prec == "f64" else 2e-6) and chk[1] <= (1e-14 if prec == "f64" else 2e-6)
    assert chk[2] == 0
    # special-unitary links move by their defect only
    Us = to_soa(sym, rounded(U, prec), L, prec, dev)
    before = from_soa(sym, Us, L)
    after = from_soa(sym, sym.reunitarise(Us, L), L)
    assert np.abs(after - before).max() <= (1e-15 if prec == "f64" else 4e-7)
    # non-finite input stays non-finite
    W = rounded(U, prec).copy()
    W[1, 2, 3, 0, 2, 1, 1] = np.nan
    Ws = to_soa(sym, W, L, prec, dev)
    sym.reunitarise(Ws, L)
    assert sym.check_links(Ws, L).cpu().numpy()[2] == 1
