"""Why the FP32 drift projects links onto SU(3): a host emulation of repeated link
updates U <- exp(dt Pi) U computed in double and rounded to float. Without projection the
unitarity defect ||U^+U - 1||_F performs a random walk and grows with the number of steps;
with the Gram-Schmidt projection of the first two rows (third row their conjugate cross
product) before each rounding it stays at float rounding. The factored force reads links
as two rows and rebuilds the third, so its error follows that defect."""
import numpy as np

import gaugegen
import oracle


def _project(U):
    r0 = U[:, 0] / np.linalg.norm(U[:, 0], axis=-1, keepdims=True)
    r1 = U[:, 1] - np.sum(np.conj(r0) * U[:, 1], axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=1)


def _defect(U):
    d = np.conj(np.swapaxes(U, -1, -2)) @ U - np.eye(3)
    return np.sqrt(np.sum(np.abs(d) ** 2, axis=(-2, -1))).max()


def test_projection_bounds_float_unitarity_drift():
    rng = np.random.default_rng(5)
    n, steps, dt = 1024, 800, 0.02
    U0 = gaugegen.haar_su3(rng, (n,))
    T = oracle.gell_mann()
    plain = U0.astype(np.complex64).astype(np.complex128)
    proj = plain.copy()
    for _ in range(steps):
        p = rng.standard_normal((n, 8))
        E = oracle.su3_exp(dt * 1j * np.einsum("na,aij->nij", p, T))
        plain = (E @ plain).astype(np.complex64).astype(np.complex128)
        proj = _project(E @ proj).astype(np.complex64).astype(np.complex128)
    d_plain, d_proj = _defect(plain), _defect(proj)
    print(f"  after {steps} steps: defect without projection {d_plain:.2e}, with projection {d_proj:.2e}")
    assert d_proj <= 1e-6
    assert d_plain > 5 * d_proj
    # the projection is a retraction: a special-unitary matrix is left unchanged
    assert np.abs(_project(U0) - U0).max() <= 1e-14
