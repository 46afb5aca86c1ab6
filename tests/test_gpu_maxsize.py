"""The largest lattice the library accepts (V/2 = 2^24 sites per parity, 64^3 x 128,
134,217,728 links), FP32 and FP64: force on sampled links against the FP64 oracle and
the fused action against the separate action kernel. Exercises the 32-bit buffer
offsets (in FP64 the last element plane of a link block starts 2 GiB into it) and the
workspace carving at their limits."""
import numpy as np
import pytest
import torch

import oracle

from gpu_util import device, force_errors

pytestmark = pytest.mark.gpu

L = (64, 64, 64, 128)
U0, BETA = 0.8677, 3.0


def _gell_mann(dev):
    return torch.from_numpy(oracle.gell_mann()).to(dev)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_force_at_the_size_limit(prec):
    import paper_1808_02281_amd as sym

    dev = device()
    Lx, Ly, Lz, Lt = L
    T = _gell_mann(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(12345)
    cdt = torch.complex64 if prec == "f32" else torch.complex128
    aos = torch.empty((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=cdt, device=dev)
    step = 8
    for t0 in range(0, Lt, step):  # near-thermal links, eps 0.25, generated slab by slab on the device
        r = torch.randn((step, Lz, Ly, Lx, 4, 8), generator=gen, device=dev, dtype=torch.float64)
        H = 0.25 * torch.einsum("...a,aij->...ij", r.to(torch.complex128), T)
        aos[t0:t0 + step] = torch.linalg.matrix_exp(1j * H).to(cdt)
        del r, H
    U = sym.pack(aos, L)
    F, S = sym.force(U, L, U0, BETA, with_action=True)
    S_act = sym.action(U, L, U0, BETA)
    torch.cuda.synchronize()
    # two FP32 evaluations (staple identity in the force pass, 34 loops per site in the
    # action kernel), both accumulated in FP64; they agree to FP32 rounding of the traces
    rel = abs(S[0].item() - S_act[0].item()) / abs(S_act[0].item())
    print(f"  64^3x128 {prec}: fused action vs action kernel {rel:.2e}", flush=True)
    assert rel <= (1e-6 if prec == "f32" else 1e-12)

    V = Lx * Ly * Lz * Lt
    rng = np.random.default_rng(7)
    sites = np.concatenate([rng.integers(0, V, 48), [0, V - 1, V // 2, V // 2 - 1]])
    mus = np.concatenate([rng.integers(0, 4, 48), [0, 3, 1, 2]]).astype(np.int32)
    Gd = sym.unpack(F, L)
    del F
    # the sampled forces, and the links on the host in FP64 for the oracle
    t_, z_, y_, x_ = np.unravel_index(sites, (Lt, Lz, Ly, Lx))
    G = Gd[torch.as_tensor(t_), torch.as_tensor(z_), torch.as_tensor(y_), torch.as_tensor(x_),
           torch.as_tensor(mus.astype(np.int64))].cpu().numpy().astype(np.complex128)
    del Gd, U
    Uh = aos.cpu().numpy().astype(np.complex128)
    del aos
    c, _ = oracle.coeffs(U0)
    Gref = oracle.force_links(Uh, L, c, BETA, sites, mus)
    e = force_errors(G, Gref)
    print(f"  64^3x128 {prec}: max {e[0]:.2e} rms {e[1]:.2e}", flush=True)
    assert e[0] <= (1e-5 if prec == "f32" else 1e-12)
    del Uh
    sym.release_workspaces()
    torch.cuda.empty_cache()
