"""Wilson-clover fermion force on the GPU against the FP64 oracle: the spinor layout
kernels, the force on every link of small lattices (several tiles and a ragged tail)
with and without the clover term, and sampled links of the 32^3x64 workload."""
import numpy as np
import pytest
import torch

import gaugegen
import oracle

from gpu_util import device, force_errors, from_soa, rounded, to_soa

pytestmark = pytest.mark.gpu

KAPPA, CSW = 0.1242, 1.37
TOL = {"f64": 1e-12, "f32": 1e-5}
SHAPES = [(4, 4, 4, 4), (6, 6, 6, 8), (8, 8, 8, 8)]


@pytest.fixture(scope="module")
def sym():
    import paper_1808_02281_amd as m

    device()
    return m


def _spinor_np(L, seed, prec):
    rng = np.random.default_rng(seed)
    shape = (L[3], L[2], L[1], L[0], 4, 3)
    return rounded(rng.standard_normal(shape) + 1j * rng.standard_normal(shape), prec)


def _to_dev_spinor(sym, X, L, prec):
    t = torch.from_numpy(np.ascontiguousarray(X)).to(torch.complex128 if prec == "f64" else torch.complex64)
    return sym.pack_spinor(t.to(device()), L)


def test_spinor_layout_round_trip(sym):
    L = (6, 4, 4, 6)
    X = _spinor_np(L, 1, "f64")
    S = _to_dev_spinor(sym, X, L, "f64")
    # the layout: field[p][3*spin + colour][cb]
    V = int(np.prod(L))
    flat = X.reshape(V, 12)
    t, z, y, x = np.meshgrid(*[np.arange(L[a]) for a in (3, 2, 1, 0)], indexing="ij")
    par = ((x + y + z + t) & 1).reshape(V)
    want = np.zeros((2, 12, V // 2), dtype=np.complex128)
    want[par, :, np.arange(V) >> 1] = flat
    got = S.cpu().numpy()
    np.testing.assert_array_equal(got[..., 0] + 1j * got[..., 1], want)
    np.testing.assert_array_equal(sym.unpack_spinor(S, L).cpu().numpy(), X)


@pytest.mark.parametrize("csw", [0.0, CSW])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("L", SHAPES)
def test_wilson_force_against_oracle(sym, L, prec, csw):
    U = rounded(gaugegen.near_thermal_links(L, 0.35, 40), prec)
    X, Y = _spinor_np(L, 41, prec), _spinor_np(L, 42, prec)
    dev = device()
    G = sym.wilson_force(to_soa(sym, U, L, prec, dev), _to_dev_spinor(sym, X, L, prec),
                         _to_dev_spinor(sym, Y, L, prec), L, KAPPA, csw)
    Go = oracle.wilson_force(U, X, Y, L, KAPPA, csw)
    e = force_errors(from_soa(sym, G, L), Go)
    print(f"  {L} {prec} csw={csw}: max {e[0]:.2e} rms {e[1]:.2e}")
    assert e[0] <= TOL[prec]


def test_wilson_force_zero_vectors(sym):
    L = (4, 4, 4, 6)
    U = gaugegen.haar_links(L, 43)
    Z = np.zeros((L[3], L[2], L[1], L[0], 4, 3), dtype=np.complex128)
    Zs = _to_dev_spinor(sym, Z, L, "f64")
    G = sym.wilson_force(to_soa(sym, U, L, "f64", device()), Zs, Zs, L, KAPPA, CSW)
    assert torch.count_nonzero(G).item() == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_wilson_force_32x32x32x64_sampled(sym, prec):
    L = gaugegen.CONFIGS["thermal_32x32x32x64"]["L"]
    U = rounded(gaugegen.make_config("thermal_32x32x32x64"), prec)
    X, Y = _spinor_np(L, 44, prec), _spinor_np(L, 45, prec)
    G = sym.wilson_force(to_soa(sym, U, L, prec, device()), _to_dev_spinor(sym, X, L, prec),
                         _to_dev_spinor(sym, Y, L, prec), L, KAPPA, CSW)
    V = int(np.prod(L))
    rng = np.random.default_rng(46)
    links = rng.choice(4 * V, 4 * V // 20, replace=False)  # 5% of the links
    sites, mus = links // 4, (links % 4).astype(np.int32)
    Go = oracle.wilson_force_links(U, X, Y, L, KAPPA, CSW, sites, mus)
    Gs = from_soa(sym, G, L).reshape(V, 4, 3, 3)[sites, mus]
    e = force_errors(Gs, Go)
    print(f"  32^3x64 {prec}: max {e[0]:.2e} rms {e[1]:.2e}")
    assert e[0] <= TOL[prec]


def test_graph_replay_matches_eager(sym):
    L = (6, 6, 6, 8)
    U = rounded(gaugegen.near_thermal_links(L, 0.35, 47), "f32")
    X, Y = _spinor_np(L, 48, "f32"), _spinor_np(L, 49, "f32")
    dev = device()
    Us = to_soa(sym, U, L, "f32", dev)
    Xs, Ys = _to_dev_spinor(sym, X, L, "f32"), _to_dev_spinor(sym, Y, L, "f32")
    eager = sym.wilson_force(Us, Xs, Ys, L, KAPPA, CSW)
    out = torch.empty_like(Us)
    sym.wilson_force(Us, Xs, Ys, L, KAPPA, CSW, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sym.wilson_force(Us, Xs, Ys, L, KAPPA, CSW, out=out)
    for rep in range(3):
        out.zero_()
        sym.wilson_force(Us, Ys, Xs, L, KAPPA, 0.0)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep}"
