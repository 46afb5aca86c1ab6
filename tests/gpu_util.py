"""Helpers shared by the GPU tests: moving fields to the device, error norms, and a
numpy statement of the even-odd layout used to check the pack kernel."""
import numpy as np
import torch

import oracle


def device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def cdtype(prec):
    return torch.complex128 if prec == "f64" else torch.complex64


def rounded(U, prec):
    """The links the kernel actually sees, promoted exactly back to complex128."""
    return U if prec == "f64" else U.astype(np.complex64).astype(np.complex128)


def to_soa(sym, U, L, prec, dev):
    aos = torch.from_numpy(np.ascontiguousarray(U)).to(cdtype(prec)).to(dev)
    return sym.pack(aos, L)


def from_soa(sym, F, L):
    return sym.unpack(F, L).cpu().numpy().astype(np.complex128)


def force_errors(G, Gref):
    """(global max relative, rms relative, worst per-link relative) in the Frobenius norm:
    max_links |G - Gref|_F / max_links |Gref|_F is the gated figure."""
    d = np.sqrt(np.sum(np.abs(G - Gref) ** 2, axis=(-2, -1)))
    r = np.sqrt(np.sum(np.abs(Gref) ** 2, axis=(-2, -1)))
    gmax = d.max() / r.max()
    rms = np.sqrt(np.mean(d ** 2)) / np.sqrt(np.mean(r ** 2))
    worst = np.max(d / np.maximum(r, 1e-300))
    return gmax, rms, worst


def soa_reference(U, L):
    """numpy statement of the SoA even-odd layout: (4, 2, 9, V/2, 2) reals."""
    Lx, Ly, Lz, Lt = L
    V = Lx * Ly * Lz * Lt
    flat = U.reshape(V, 4, 9)
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    par = ((x + y + z + t) & 1).reshape(V)
    cb = np.arange(V) >> 1
    out = np.zeros((4, 2, 9, V // 2), dtype=np.complex128)
    for mu in range(4):
        out[mu, par, :, cb] = flat[:, mu, :]
    return np.stack([out.real, out.imag], axis=-1)


def lie_derivative(G):
    return oracle.lie_derivative(G)
