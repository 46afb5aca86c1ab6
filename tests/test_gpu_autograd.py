"""The action as a differentiable torch function whose backward is the force kernel.

Links are parametrised as U = exp(i omega.T) U0 with torch ops; gradients with respect
to omega come from the hand-written backward (2 G U per link) through torch's chain
rule, and are checked against finite differences of the GPU action, torch's gradcheck,
and the oracle's -2i tr(T_a G) at omega = 0."""
import numpy as np
import pytest
import torch

import gaugegen
import oracle

from gpu_util import device

pytestmark = pytest.mark.gpu

U0, BETA = gaugegen.U0, gaugegen.BETA


@pytest.fixture(scope="module")
def sym():
    import paper_1808_02281_amd as m

    device()
    m.set_force_algorithm("auto")
    return m


def _links(omega, U0c, T):
    H = torch.einsum("...a,aij->...ij", omega.to(T.dtype), T)
    return torch.linalg.matrix_exp(1j * H) @ U0c


def _setup(L, eps, seed, dtype=torch.complex128):
    dev = device()
    U = gaugegen.near_thermal_links(L, eps, seed)
    T = torch.from_numpy(oracle.gell_mann()).to(dtype).to(dev)
    return U, torch.from_numpy(U).to(dtype).to(dev), T


def _action_of_omega(sym, L, U0c, T):
    from paper_1808_02281_amd import autograd as ag

    def f(omega):
        return ag.symanzik_action(ag.pack(_links(omega, U0c, T).contiguous(), L), L, U0, BETA)

    return f


def test_gradcheck_4x4x4x4(sym):
    L = (4, 4, 4, 4)
    _, U0c, T = _setup(L, 0.4, 21)
    f = _action_of_omega(sym, L, U0c, T)
    omega = (0.05 * torch.randn(gaugegen.field_shape(L, (4, 8)), dtype=torch.float64, device=device())).requires_grad_()
    assert torch.autograd.gradcheck(f, (omega,), eps=1e-6, atol=1e-6, rtol=1e-5, fast_mode=True)


def test_autograd_vs_finite_differences_8x8x8x8(sym):
    L = (8, 8, 8, 8)
    _, U0c, T = _setup(L, 0.3, 22)
    f = _action_of_omega(sym, L, U0c, T)
    gen = torch.Generator(device="cpu").manual_seed(3)
    omega = 0.1 * torch.randn(gaugegen.field_shape(L, (4, 8)), dtype=torch.float64, generator=gen).to(device())
    w = omega.clone().requires_grad_()
    f(w).backward()
    g = w.grad.reshape(-1)
    flat = omega.reshape(-1)
    rng = np.random.default_rng(4)
    eps = 1e-5
    worst = 0.0
    for i in rng.integers(0, flat.numel(), 64):
        i = int(i)
        vals = []
        for s in (1, -1):
            o = flat.clone()
            o[i] += s * eps
            vals.append(f(o.reshape(omega.shape)).item())
        fd = (vals[0] - vals[1]) / (2 * eps)
        worst = max(worst, abs(fd - g[i].item()) / max(1.0, abs(g[i].item())))
    print(f"  worst autograd vs finite-difference error: {worst:.2e}")
    assert worst <= 1e-6


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-11), (torch.complex64, 1e-5)])
def test_gradient_at_zero_matches_oracle_24x24x24x48(sym, dtype, tol):
    """dS/domega at omega = 0 through torch autograd against the oracle's Lie derivative
    -2i tr(T_a G) on 5% of the links (132,710), drawn without replacement."""
    cfg = gaugegen.CONFIGS["thermal_24x24x24x48"]
    L = cfg["L"]
    U, U0c, T = _setup(L, cfg["eps"], cfg["seed"], dtype)
    f = _action_of_omega(sym, L, U0c, T)
    omega = torch.zeros(gaugegen.field_shape(L, (4, 8)), dtype=torch.float64, device=device(), requires_grad=True)
    f(omega).backward()
    V = int(np.prod(L))
    rng = np.random.default_rng(cfg["fd_seed"])
    links = rng.choice(4 * V, 4 * V // 20, replace=False)  # 5% of the links
    sites, mus = links // 4, links % 4
    Ur = U if dtype == torch.complex128 else U.astype(np.complex64).astype(np.complex128)
    c, _ = oracle.coeffs(U0)
    d_ref = oracle.lie_derivative(oracle.force_links(Ur, L, c, BETA, sites, mus))
    d_gpu = omega.grad.reshape(V, 4, 8)[torch.from_numpy(sites).to(device()), torch.from_numpy(mus).to(device())]
    d_gpu = d_gpu.cpu().numpy()
    err = np.abs(d_gpu - d_ref).max() / np.abs(d_ref).max()
    print(f"  {dtype}: max |dS/domega - oracle| / max |oracle| = {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-6)])
def test_forward_value_with_and_without_grad(sym, dtype, tol):
    """With a backward possible the forward takes S from the force kernels' fused
    action; without, from the action kernel: the same S (and the oracle's)."""
    from paper_1808_02281_amd import autograd as ag

    L = (6, 6, 6, 8)
    U = gaugegen.near_thermal_links(L, 0.3, 23)
    Us = ag.pack(torch.from_numpy(U).to(dtype).to(device()), L)
    with torch.no_grad():
        s0 = ag.symanzik_action(Us, L, U0, BETA).item()
    x = Us.clone().requires_grad_(True)
    S = ag.symanzik_action(x, L, U0, BETA)
    s1 = S.item()
    S.backward()
    Ur = U if dtype == torch.complex128 else U.astype(np.complex64).astype(np.complex128)
    c, _ = oracle.coeffs(U0)
    s_ref = oracle.action(Ur, L, c, BETA)[0]
    assert abs(s1 - s0) <= tol * abs(s0)
    assert abs(s1 - s_ref) <= tol * abs(s_ref)
    assert x.grad is not None and torch.isfinite(x.grad).all()
