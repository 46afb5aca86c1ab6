"""Write the stored expected values under tests/golden/ from the FP64 CPU oracle only.

leapfrog_24x24x24x48.json: a 10-step leapfrog trajectory (dt = 0.02) on the
24^3x48 near-thermal workload (eps = 0.3, link seed 3, momentum seed 4, u0 = 0.8677,
beta = 3) computed by the oracle's plain position-momentum-position leapfrog
(half kick, exact exponential drift, half kick; arXiv:1808.02281 Sec. II for the
force, Pi-dot = -G and U-dot = Pi U for the dynamics). Stores H before and after,
dH, and 32 sampled links of U and P at the end.

Run:  python tests/golden/make_golden.py   (about 5-10 minutes on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gaugegen  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def leapfrog_24():
    cfg = gaugegen.CONFIGS["thermal_24x24x24x48"]
    L = cfg["L"]
    U = gaugegen.near_thermal_links(L, cfg["eps"], cfg["seed"])
    P = gaugegen.momenta(L, cfg["momenta_seed"])
    c, _ = oracle.coeffs(gaugegen.U0)
    t0 = time.time()
    U1, P1, H0, H1 = oracle.leapfrog(U, P, L, c, gaugegen.BETA, 0.02, 10)
    rng = np.random.default_rng(12)
    V = int(np.prod(L))
    sites = rng.integers(0, V, 32)
    mus = rng.integers(0, 4, 32)
    Uf = U1.reshape(V, 4, 3, 3)
    Pf = P1.reshape(V, 4, 3, 3)
    out = {
        "what": "10-step leapfrog, dt=0.02, on the 24^3x48 near-thermal workload (FP64 CPU oracle)",
        "L": list(L), "eps": cfg["eps"], "link_seed": cfg["seed"], "momentum_seed": cfg["momenta_seed"],
        "u0": gaugegen.U0, "beta": gaugegen.BETA, "dt": 0.02, "nsteps": 10,
        "H_start": H0, "H_end": H1, "dH": H1 - H0,
        "sample_sites": sites.tolist(), "sample_mus": mus.tolist(),
        "U_end_re": Uf[sites, mus].real.tolist(), "U_end_im": Uf[sites, mus].imag.tolist(),
        "P_end_re": Pf[sites, mus].real.tolist(), "P_end_im": Pf[sites, mus].imag.tolist(),
        "oracle_seconds": time.time() - t0, "oracle_threads": oracle.num_threads(),
    }
    with open(os.path.join(HERE, "leapfrog_24x24x24x48.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"H_start {H0!r} H_end {H1!r} dH {H1 - H0!r} ({out['oracle_seconds']:.0f} s)")


if __name__ == "__main__":
    leapfrog_24()
