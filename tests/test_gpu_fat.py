"""Fat-link smearing (asqtad / HISQ) and its path force on the GPU against the FP64 oracle:
fat and Naik links, the pulled-back gradient and the thin-link force, element by
element on small lattices (several tiles and a ragged tail), on sampled links of the
32^3x64 workload, through autograd, and through a two-level smearing chain."""
import numpy as np
import pytest
import torch

import gaugegen
import oracle

from gpu_util import device, force_errors, from_soa, rounded, to_soa

pytestmark = pytest.mark.gpu

C_ASQTAD = (5 / 8, -1 / 16, 1 / 64, -1 / 384, -1 / 16, -1 / 24)
C_GENERIC = (0.61, -0.071, 0.013, -0.0029, -0.055, -0.043)
TOL = {"f64": 1e-12, "f32": 1e-5}

SHAPES = [(4, 4, 4, 4), (6, 6, 6, 8), (8, 8, 8, 8)]


@pytest.fixture(scope="module")
def sym():
    import paper_1808_02281_amd as m

    device()
    return m


def _rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _inputs(L, seed, prec):
    rng = np.random.default_rng(seed)
    U = rounded(gaugegen.near_thermal_links(L, 0.35, seed), prec)
    GV = rounded(_rand_c(rng, U.shape), prec)
    GW = rounded(_rand_c(rng, U.shape), prec)
    return U, GV, GW


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("L", SHAPES)
def test_fat_links_against_oracle(sym, L, prec):
    U, _, _ = _inputs(L, 21, prec)
    dev = device()
    V, W = sym.fat_links(to_soa(sym, U, L, prec, dev), L, C_GENERIC)
    Vo, Wo = oracle.fat_links(U, L, C_GENERIC)
    ev, ew = _rel(from_soa(sym, V, L), Vo), _rel(from_soa(sym, W, L), Wo)
    print(f"  {L} {prec}: V {ev:.2e}  W {ew:.2e}")
    assert ev <= TOL[prec] and ew <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("L", SHAPES)
def test_fat_gradient_and_force_against_oracle(sym, L, prec):
    U, GV, GW = _inputs(L, 22, prec)
    dev = device()
    Us = to_soa(sym, U, L, prec, dev)
    GVs, GWs = to_soa(sym, GV, L, prec, dev), to_soa(sym, GW, L, prec, dev)
    g = from_soa(sym, sym.fat_force(Us, L, C_ASQTAD, GVs, GWs, mode="grad"), L)
    go = oracle.fat_grad(U, L, C_ASQTAD, GV, GW)
    G = from_soa(sym, sym.fat_force(Us, L, C_ASQTAD, GVs, GWs, mode="force"), L)
    Go = oracle.fat_force_from_grad(U, go)
    eg = _rel(g, go)
    ef = force_errors(G, Go)
    print(f"  {L} {prec}: grad {eg:.2e}  force max {ef[0]:.2e} rms {ef[1]:.2e}")
    assert eg <= TOL[prec] and ef[0] <= TOL[prec]


def test_fat_gradient_without_naik(sym):
    L = (6, 6, 6, 8)
    U, GV, _ = _inputs(L, 23, "f64")
    dev = device()
    Us, GVs = to_soa(sym, U, L, "f64", dev), to_soa(sym, GV, L, "f64", dev)
    g = from_soa(sym, sym.fat_force(Us, L, C_GENERIC, GVs, None, mode="grad"), L)
    assert _rel(g, oracle.fat_grad(U, L, C_GENERIC, GV, None)) <= 1e-12


def test_fat_single_classes(sym):
    """Each coefficient class alone (a dropped or swapped class on either side fails)."""
    L = (4, 4, 6, 4)
    U, GV, GW = _inputs(L, 24, "f64")
    dev = device()
    Us, GVs, GWs = (to_soa(sym, X, L, "f64", dev) for X in (U, GV, GW))
    for k in range(6):
        c = [0.0] * 6
        c[k] = 1.0
        V, W = sym.fat_links(Us, L, c)
        Vo, Wo = oracle.fat_links(U, L, c)
        np.testing.assert_allclose(from_soa(sym, V, L), Vo, atol=1e-12)
        np.testing.assert_allclose(from_soa(sym, W, L), Wo, atol=1e-12)
        g = from_soa(sym, sym.fat_force(Us, L, c, GVs, GWs, mode="grad"), L)
        np.testing.assert_allclose(g, oracle.fat_grad(U, L, c, GV, GW), atol=1e-11)


def test_unit_field(sym):
    L = (4, 4, 4, 6)
    U = gaugegen.unit_links(L)
    V, W = sym.fat_links(to_soa(sym, U, L, "f64", device()), L, C_ASQTAD)
    c1, c3, c5, c7, cL, cN = C_ASQTAD
    n = c1 + 6 * c3 + 24 * c5 + 48 * c7 + 6 * cL
    np.testing.assert_allclose(from_soa(sym, V, L), n * U, atol=1e-15)
    np.testing.assert_allclose(from_soa(sym, W, L), cN * U, atol=1e-15)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fat_32x32x32x64_sampled(sym, prec):
    """The benchmark workload and launch configuration, checked on 5% of the links
    (419,430, drawn without replacement)."""
    cfg = gaugegen.CONFIGS["thermal_32x32x32x64"]
    L = cfg["L"]
    dev = device()
    U = rounded(gaugegen.make_config("thermal_32x32x32x64"), prec)
    rng = np.random.default_rng(25)
    GV = rounded(0.1 * _rand_c(rng, U.shape), prec)
    GW = rounded(0.1 * _rand_c(rng, U.shape), prec)
    Us = to_soa(sym, U, L, prec, dev)
    GVs, GWs = to_soa(sym, GV, L, prec, dev), to_soa(sym, GW, L, prec, dev)
    V, W = sym.fat_links(Us, L, C_ASQTAD)
    g = sym.fat_force(Us, L, C_ASQTAD, GVs, GWs, mode="grad")
    del GVs, GWs
    nV = L[0] * L[1] * L[2] * L[3]
    links = rng.choice(4 * nV, 4 * nV // 20, replace=False)
    sites, mus = links // 4, (links % 4).astype(np.int32)
    Vo, Wo = oracle.fat_links_links(U, L, C_ASQTAD, sites, mus)
    go = oracle.fat_grad_links(U, L, C_ASQTAD, GV, GW, sites, mus)
    pick = lambda F: from_soa(sym, F, L).reshape(nV, 4, 3, 3)[sites, mus]
    ev, ew, eg = _rel(pick(V), Vo), _rel(pick(W), Wo), _rel(pick(g), go)
    print(f"  32^3x64 {prec}: V {ev:.2e}  W {ew:.2e}  grad {eg:.2e}")
    assert max(ev, ew, eg) <= TOL[prec]


def test_autograd_matches_oracle(sym):
    """Phi = Re sum tr(GV^+ V) + Re sum tr(GW^+ W) built in torch from fat_smear; U.grad
    is the oracle gradient in the real SoA layout."""
    L = (6, 6, 6, 8)
    U, GV, GW = _inputs(L, 26, "f64")
    dev = device()
    Us = to_soa(sym, U, L, "f64", dev).requires_grad_(True)
    GVs, GWs = to_soa(sym, GV, L, "f64", dev), to_soa(sym, GW, L, "f64", dev)
    V, W = sym.fat_smear(Us, L, C_ASQTAD)
    phi = (GVs * V).sum() + (GWs * W).sum()
    phi.backward()
    g = from_soa(sym, Us.grad.contiguous(), L)
    assert _rel(g, oracle.fat_grad(U, L, C_ASQTAD, GV, GW)) <= 1e-12


def test_gradcheck_small(sym):
    L = (4, 4, 4, 4)
    U, GV, GW = _inputs(L, 27, "f64")
    dev = device()
    Us = to_soa(sym, U, L, "f64", dev).requires_grad_(True)
    GVs = to_soa(sym, GV, L, "f64", dev)

    def f(x):
        V, W = sym.fat_smear(x, L, C_GENERIC)
        return (GVs * V).sum() + (W * W).sum()

    assert torch.autograd.gradcheck(f, (Us,), eps=1e-6, atol=1e-7, rtol=1e-6, fast_mode=True)


def test_two_level_chain_finite_differences(sym):
    """HISQ-like chain: V = F[U] (fat7 coefficients), Y = V / |V| (a smooth, non-unitary
    map written in torch), X, N = F[Y] (asqtad coefficients); the chained gradient
    (two pull-backs by the path-force kernels plus torch's for the middle step) matches
    central differences of the scalar along random complex directions."""
    L = (4, 4, 4, 4)
    U, GV, GW = _inputs(L, 28, "f64")
    dev = device()
    Us = to_soa(sym, U, L, "f64", dev)
    GVs, GWs = to_soa(sym, GV, L, "f64", dev), to_soa(sym, GW, L, "f64", dev)
    fat7 = (1 / 8, -1 / 16, 1 / 64, -1 / 384, 0.0, 0.0)

    def phi(x):
        V, _ = sym.fat_smear(x, L, fat7)
        Y = V / (1.0 + (V * V).sum(dim=(2, 4), keepdim=True))
        X, N = sym.fat_smear(Y.contiguous(), L, C_ASQTAD)
        return (GVs * X).sum() + (GWs * N).sum()

    x = Us.clone().requires_grad_(True)
    phi(x).backward()
    grad = x.grad.detach()
    rng = np.random.default_rng(29)
    for _ in range(3):
        E = torch.from_numpy(rng.standard_normal(Us.shape)).to(dev)
        eps = 1e-5
        with torch.no_grad():
            fd = (phi(Us + eps * E) - phi(Us - eps * E)).item() / (2 * eps)
        an = (grad * E).sum().item()
        assert abs(fd - an) <= 1e-7 * abs(an), (fd, an)


def test_graph_replay_matches_eager(sym):
    """The path force is plain kernel launches on the caller's stream: captured once into
    a HIP graph, every replay (with eager work in between) reproduces the eager result."""
    L = (6, 6, 6, 8)
    U, GV, GW = _inputs(L, 30, "f32")
    dev = device()
    Us, GVs, GWs = (to_soa(sym, X, L, "f32", dev) for X in (U, GV, GW))
    eager = sym.fat_force(Us, L, C_ASQTAD, GVs, GWs, mode="force")
    out = torch.empty_like(Us)
    sym.fat_force(Us, L, C_ASQTAD, GVs, GWs, mode="force", out=out)  # warm the workspace cache
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sym.fat_force(Us, L, C_ASQTAD, GVs, GWs, mode="force", out=out)
    for rep in range(3):
        out.zero_()
        sym.fat_links(Us, L, C_GENERIC)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep}"


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_reuse_of_forward_intermediates(sym, prec):
    """fat_force with reuse_links on the workspace that fat_links filled gives bitwise
    the result of the full call, in both output modes."""
    L = (6, 6, 6, 8)
    U, GV, GW = _inputs(L, 31, prec)
    dev = device()
    Us, GVs, GWs = (to_soa(sym, X, L, prec, dev) for X in (U, GV, GW))
    ws = sym.new_fat_workspace(L, sym.prec_of(Us.dtype), dev)
    for mode in ("grad", "force"):
        full = sym.fat_force(Us, L, C_ASQTAD, GVs, GWs, mode=mode)
        sym.fat_links(Us, L, C_ASQTAD, ws=ws)
        again = sym.fat_force(Us, L, C_ASQTAD, GVs, GWs, mode=mode, ws=ws, reuse_links=True)
        assert torch.equal(full, again), mode
    with pytest.raises(ValueError):
        sym.fat_force(Us, L, C_ASQTAD, GVs, GWs, reuse_links=True)

