"""Molecular dynamics on the GPU: leapfrog parity with the oracle, finite differences of
the action against the GPU force on the 24^3x48 workload, and the energy change of a
10-step trajectory against the stored oracle value."""
import json
import os

import numpy as np
import pytest
import torch

import gaugegen
import oracle

from gpu_util import device, force_errors, from_soa, rounded, to_soa

pytestmark = pytest.mark.gpu

U0, BETA = gaugegen.U0, gaugegen.BETA
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "leapfrog_24x24x24x48.json")


@pytest.fixture(scope="module")
def sym():
    import paper_1808_02281_amd as m

    device()
    m.set_force_algorithm("auto")
    return m


@pytest.fixture(scope="module")
def c():
    return oracle.coeffs(U0)[0]


@pytest.mark.parametrize("alg", ["direct", "factored"])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_leapfrog_parity_small(sym, c, alg, prec, tol):
    print(f"case leapfrog 4x4x6x4 {prec} {alg}", flush=True)
    sym.set_force_algorithm(alg)
    L = (4, 4, 6, 4)
    U = rounded(gaugegen.near_thermal_links(L, 0.3, 3), prec)
    P = rounded(gaugegen.momenta(L, 4), prec)
    U1, P1, H0, H1 = oracle.leapfrog(U, P, L, c, BETA, 0.05, 4)
    dev = device()
    Us, Ps = to_soa(sym, U, L, prec, dev), to_soa(sym, P, L, prec, dev)
    H = sym.md_leapfrog(Us, Ps, L, U0, BETA, 0.05, 4).cpu().numpy()
    dU = np.abs(from_soa(sym, Us, L) - U1).max()
    dP = np.abs(from_soa(sym, Ps, L) - P1).max() / np.abs(P1).max()
    print(f"  |dU| {dU:.2e} |dP|/|P| {dP:.2e} H0 {abs(H[0]-H0)/H0:.2e} H1 {abs(H[1]-H1)/H1:.2e} "
          f"dH gpu {H[1]-H[0]:.6e} oracle {H1-H0:.6e}")
    assert dU <= tol and dP <= tol
    assert abs(H[0] - H0) <= tol * H0 and abs(H[1] - H1) <= tol * H1
    sym.set_force_algorithm("auto")


def test_leapfrog_zero_steps_and_reversibility(sym):
    L = (4, 4, 4, 4)
    dev = device()
    U = gaugegen.near_thermal_links(L, 0.3, 5)
    P = gaugegen.momenta(L, 6)
    Us, Ps = to_soa(sym, U, L, "f64", dev), to_soa(sym, P, L, "f64", dev)
    U_in, P_in = Us.clone(), Ps.clone()
    H = sym.md_leapfrog(Us, Ps, L, U0, BETA, 0.05, 0).cpu().numpy()
    assert H[0] == H[1]
    assert torch.equal(Us, U_in) and torch.equal(Ps, P_in)
    sym.md_leapfrog(Us, Ps, L, U0, BETA, 0.05, 6)
    Ps.neg_()
    sym.md_leapfrog(Us, Ps, L, U0, BETA, 0.05, 6)
    assert torch.abs(Us - U_in).max().item() < 1e-12
    assert torch.abs(Ps + P_in).max().item() < 1e-12


@pytest.fixture(scope="module")
def cfg4():
    cfg = gaugegen.CONFIGS["thermal_24x24x24x48"]
    return cfg, gaugegen.near_thermal_links(cfg["L"], cfg["eps"], cfg["seed"])


def test_finite_differences_24x24x24x48(sym, c, cfg4):
    """dS/domega^a = -2i tr(T_a G) from the GPU force against central differences
    (eps = 1e-4, FP64) of the oracle's action restricted to the loops through the link,
    on 1000 random links and all 8 generators."""
    cfg, U = cfg4
    L = cfg["L"]
    V = int(np.prod(L))
    dev = device()
    F = sym.force(to_soa(sym, U, L, "f64", dev), L, U0, BETA)
    G = sym.unpack(F, L).reshape(V, 4, 3, 3)
    rng = np.random.default_rng(cfg["fd_seed"])
    sites = rng.integers(0, V, 1000)
    mus = rng.integers(0, 4, 1000)
    Gs = G[torch.from_numpy(sites).to(dev), torch.from_numpy(mus).to(dev)].cpu().numpy()
    d_gpu = oracle.lie_derivative(Gs)
    T = oracle.gell_mann()
    eps = 1e-4
    E = {(a, s): oracle.su3_exp(1j * s * eps * T[a]) for a in range(8) for s in (1, -1)}
    Uf = U.reshape(V, 4, 3, 3)
    worst = 0.0
    for i in range(1000):
        s, mu = int(sites[i]), int(mus[i])
        keep = Uf[s, mu].copy()
        for a in range(8):
            vals = []
            for sg in (1, -1):
                Uf[s, mu] = E[(a, sg)] @ keep
                vals.append(oracle.local_action(U, L, c, BETA, s, mu))
            Uf[s, mu] = keep
            fd = (vals[0] - vals[1]) / (2 * eps)
            err = abs(fd - d_gpu[i, a]) / max(1.0, abs(d_gpu[i]).max())
            worst = max(worst, err)
    print(f"  worst finite-difference relative error over 8000 derivatives: {worst:.2e}")
    assert worst <= 1e-6


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_trajectory_energy_change_24x24x24x48(sym, cfg4, prec):
    """10 leapfrog steps, dt = 0.02, Gaussian momenta: H and dH against the stored
    oracle trajectory (FP64 gate 1e-10 relative on H; FP32 reported with a loose bound)."""
    gold = json.load(open(GOLDEN))
    cfg, U = cfg4
    L = cfg["L"]
    P = gaugegen.momenta(L, cfg["momenta_seed"])
    dev = device()
    Us, Ps = to_soa(sym, U, L, prec, dev), to_soa(sym, P, L, prec, dev)
    H = sym.md_leapfrog(Us, Ps, L, U0, BETA, gold["dt"], gold["nsteps"]).cpu().numpy()
    dH = H[1] - H[0]
    print(f"  {prec}: H0 {H[0]:.10e} (oracle {gold['H_start']:.10e}) dH {dH:.6e} (oracle {gold['dH']:.6e})")
    if prec == "f64":
        assert abs(H[0] - gold["H_start"]) <= 1e-12 * gold["H_start"]
        assert abs(H[1] - gold["H_end"]) <= 1e-12 * gold["H_end"]
        assert abs(dH - gold["dH"]) <= 1e-6 * max(1.0, abs(gold["dH"]))
        V = int(np.prod(L))
        Ue = sym.unpack(Us, L).reshape(V, 4, 3, 3).cpu().numpy()
        idx = (np.array(gold["sample_sites"]), np.array(gold["sample_mus"]))
        ref = np.array(gold["U_end_re"]) + 1j * np.array(gold["U_end_im"])
        assert np.abs(Ue[idx] - ref).max() <= 1e-12
    else:
        assert abs(dH - gold["dH"]) <= 1e-6 * gold["H_start"]


def test_long_fp32_chain_stays_special_unitary(sym, c):
    """500 FP32 leapfrog steps on 8^4 (five trajectories of 100 steps, dt = 0.02, fresh
    Gaussian momenta each): the drift projects every updated link onto SU(3) before
    rounding, so the unitarity defect stays at float rounding, and the factored force
    (which rebuilds third rows) agrees with the direct force (which reads every
    element) and with the oracle on the drifted links at the FP32 gate."""
    L = (8, 8, 8, 8)
    dev = device()
    Us = to_soa(sym, gaugegen.near_thermal_links(L, 0.3, 21), L, "f32", dev)
    for traj in range(5):
        Ps = to_soa(sym, gaugegen.momenta(L, 100 + traj), L, "f32", dev)
        H = sym.md_leapfrog(Us, Ps, L, U0, BETA, 0.02, 100).cpu().numpy()
        assert np.isfinite(H).all()
        chk = sym.check_links(Us, L).cpu().numpy()
        print(f"  trajectory {traj}: dH {H[1] - H[0]:.3e}, max |U^+U - 1| {chk[0]:.2e}, max |det U - 1| {chk[1]:.2e}",
              flush=True)
        assert chk[0] <= 1e-6 and chk[1] <= 1e-6 and chk[2] == 0
    sym.set_force_algorithm("direct")
    Fd = from_soa(sym, sym.force(Us, L, U0, BETA), L)
    sym.set_force_algorithm("factored")
    Ff = from_soa(sym, sym.force(Us, L, U0, BETA), L)
    sym.set_force_algorithm("auto")
    Ud = from_soa(sym, Us, L)
    G_ref = oracle.force(Ud, L, c, BETA)
    e_fd = force_errors(Ff, Fd)[0]
    e_f, e_d = force_errors(Ff, G_ref)[0], force_errors(Fd, G_ref)[0]
    print(f"  after 500 steps: factored vs direct {e_fd:.2e}, factored vs oracle {e_f:.2e}, direct vs oracle {e_d:.2e}")
    assert max(e_fd, e_f, e_d) <= 1e-5
