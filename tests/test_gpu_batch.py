"""Batched force over independent lattices of uneven sizes (one persistent launch per
pass), the autotuner, and replay of a captured HIP graph of the batched call."""
import numpy as np
import pytest
import torch

import gaugegen
import oracle

from gpu_util import device, force_errors, from_soa, to_soa

pytestmark = pytest.mark.gpu

U0, BETA = gaugegen.U0, gaugegen.BETA

SHAPES = [(4, 4, 4, 4), (6, 6, 6, 8), (8, 8, 8, 8), (4, 8, 6, 10), (8, 8, 8, 16), (12, 12, 12, 12)]


@pytest.fixture(scope="module")
def sym():
    import paper_1808_02281_amd as m

    device()
    m.set_force_algorithm("factored")
    yield m
    m.set_force_algorithm("auto")


def _fields(shapes, prec, seed0=30):
    dev = device()
    return [to_soa(__import__("paper_1808_02281_amd"), gaugegen.near_thermal_links(L, 0.2 + 0.03 * i, seed0 + i), L,
                   prec, dev) for i, L in enumerate(shapes)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_equals_single_lattice_calls(sym, prec):
    Us = _fields(SHAPES, prec)
    Fs, S = sym.force_batch(Us, SHAPES, U0, BETA, with_action=True)
    for i, (U, L) in enumerate(zip(Us, SHAPES)):
        F1, S1 = sym.force(U, L, U0, BETA, with_action=True)
        assert torch.equal(Fs[i], F1), f"lattice {i} {L}"
        assert abs(S[i, 0].item() - S1[0].item()) <= 1e-12 * abs(S1[0].item())


def test_batch_against_oracle(sym):
    c, _ = oracle.coeffs(U0)
    shapes = SHAPES[:4]
    Uh = [gaugegen.near_thermal_links(L, 0.35, 50 + i) for i, L in enumerate(shapes)]
    Us = [to_soa(sym, U, L, "f64", device()) for U, L in zip(Uh, shapes)]
    Fs, S = sym.force_batch(Us, shapes, U0, BETA, with_action=True)
    for i, L in enumerate(shapes):
        G_ref = oracle.force(Uh[i], L, c, BETA)
        S_ref, W_ref = oracle.action(Uh[i], L, c, BETA)
        assert force_errors(from_soa(sym, Fs[i], L), G_ref)[0] <= 1e-12
        assert abs(S[i, 0].item() - S_ref) <= 1e-12 * abs(S_ref)
        np.testing.assert_allclose(S[i, 1:].cpu().numpy(), W_ref, rtol=1e-12)


def test_batch_larger_than_one_launch(sym):
    """70 lattices: two launches per pass (64 + 6)."""
    shapes = [(4, 4, 4, 4)] * 66 + [(4, 4, 6, 4)] * 4
    Us = _fields(shapes, "f32", seed0=100)
    Fs, S = sym.force_batch(Us, shapes, U0, BETA, with_action=True)
    for i in (0, 63, 64, 69):
        F1, S1 = sym.force(Us[i], shapes[i], U0, BETA, with_action=True)
        assert torch.equal(Fs[i], F1)
        assert abs(S[i, 0].item() - S1[0].item()) <= 1e-12 * abs(S1[0].item())


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_autotune_keeps_results(sym, prec):
    """The autotuner times 48 schedules (256 or 128 links per workgroup, three occupancy
    caps, one workgroup per tile or 2048/1024/512 persistent workgroups, two tile
    orders); its last candidate is 512 persistent workgroups of 128 links at one
    workgroup per CU. The default schedule, the last candidate and the schedule it keeps
    give bitwise the same forces, and every candidate is logged."""
    Us = _fields(SHAPES, prec, seed0=7)
    F0 = sym.force_batch(Us, SHAPES, U0, BETA)
    Fp = [torch.empty_like(U) for U in Us]
    best, log = sym.batch_autotune(Us, SHAPES, U0, BETA, out=Fp)
    space = {(g, o, l, d) for g in (0, 2048, 1024, 512) for o in (0, 1) for l in (256, 128) for d in (0, -1, 96)}
    assert len(log) == 48
    assert {tuple(c.values()) for c, _ in log} == space
    assert all(ms > 0 for _, ms in log)
    assert tuple(best.values()) in space
    assert min(ms for _, ms in log) == [ms for c, ms in log if c == best][0]
    print(f"  best schedule {best}; default-like {[ms for c, ms in log if c == dict(grid=0, order=1, links=256, lds_kib=-1)]}")
    F1 = sym.force_batch(Us, SHAPES, U0, BETA)
    for a, b, c in zip(F0, F1, Fp):
        assert torch.equal(a, b)
        assert torch.equal(a, c)


def test_graph_replay_matches_eager(sym):
    Us = _fields(SHAPES, "f32", seed0=11)
    F_eager, S_eager = sym.force_batch(Us, SHAPES, U0, BETA, with_action=True)
    Fs = [torch.empty_like(U) for U in Us]
    S = torch.empty((len(Us), 4), dtype=torch.float64, device=device())
    sym.force_batch(Us, SHAPES, U0, BETA, with_action=True, out=Fs, S_out=S)  # warm the workspace cache
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sym.force_batch(Us, SHAPES, U0, BETA, with_action=True, out=Fs, S_out=S)
    for rep in range(3):
        for F in Fs:
            F.zero_()
        S.zero_()
        # eager work and a synchronisation between replays
        sym.force(Us[0], SHAPES[0], U0, BETA)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(Fs, F_eager):
            assert torch.equal(a, b), f"replay {rep}"
        assert torch.equal(S, S_eager), f"replay {rep}"
