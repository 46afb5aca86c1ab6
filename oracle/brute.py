"""Brute-force numpy enumeration of the Symanzik loop sum, for tiny lattices only.

Test infrastructure. Written independently of ``sym_oracle.c``: every loop of
eq. (18_3_27_30) is spelled out term by term as a product of shifted link fields
(``numpy.roll``), and summed as in eq. (18_6_4_1). It pins the oracle's loop set,
orientation and coefficients; it is far too slow to be anything but a checker.

Field layout: complex128 ``(Lt, Lz, Ly, Lx, 4, 3, 3)``; axis a of the lattice
(0=x .. 3=t) is array axis ``3 - a``.
"""
import numpy as np


def _shift(F, axis, k):
    """F(n + k*axis_hat) as a field over n (periodic)."""
    return np.roll(F, -k, axis=3 - axis)


def _link(U, mu, offset):
    """Field n -> U_{n+offset, mu} for forward mu (offset is a 4-vector)."""
    F = U[..., mu, :, :]
    for a in range(4):
        if offset[a]:
            F = _shift(F, a, offset[a])
    return F


def _walk(U, dirs):
    """Field n -> product of links along the signed step list ``dirs`` starting at n.

    Steps are (axis, +1/-1). A backward step from m along axis a uses U_{m-a, a}^dagger.
    """
    pos = [0, 0, 0, 0]
    P = None
    for a, s in dirs:
        if s > 0:
            M = _link(U, a, pos)
            pos[a] += 1
        else:
            pos[a] -= 1
            M = np.conj(np.swapaxes(_link(U, a, pos), -1, -2))
        P = M if P is None else P @ M
    return P


def loop_sums(U):
    """W_plaq, W_rect, W_cube: sums over sites of Re tr of every loop of eq. (18_3_27_30)."""
    W = [0.0, 0.0, 0.0]
    # plaquettes U_{n,mu} U_{n+mu,nu} U_{n+mu+nu,-mu} U_{n+nu,-nu}, mu < nu
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = _walk(U, [(mu, 1), (nu, 1), (mu, -1), (nu, -1)])
            W[0] += np.trace(P, axis1=-2, axis2=-1).real.sum()
    # rectangles: two steps along mu, one along nu, back: mu != nu
    for mu in range(4):
        for nu in range(4):
            if nu == mu:
                continue
            P = _walk(U, [(mu, 1), (mu, 1), (nu, 1), (mu, -1), (mu, -1), (nu, -1)])
            W[1] += np.trace(P, axis1=-2, axis2=-1).real.sum()
    # cube loops: mu, +-nu, +-rho, -mu, -+nu, -+rho with mu < nu < rho
    for mu in range(4):
        for nu in range(mu + 1, 4):
            for rho in range(nu + 1, 4):
                for s in (1, -1):
                    for t in (1, -1):
                        P = _walk(U, [(mu, 1), (nu, s), (rho, t), (mu, -1), (nu, -s), (rho, -t)])
                        W[2] += np.trace(P, axis1=-2, axis2=-1).real.sum()
    return np.array(W)


def action(U, c, beta):
    """S_G = beta/3 sum_n sum_P c_P [3 - Re tr P_n] with per-site counts 6, 12, 16."""
    V = U.shape[0] * U.shape[1] * U.shape[2] * U.shape[3]
    W = loop_sums(U)
    counts = np.array([6, 12, 16])
    return beta / 3.0 * float(np.sum(np.asarray(c) * (3.0 * counts * V - W))), W


def wilson_action(U, beta):
    """Textbook Wilson plaquette action beta * sum_{x, mu<nu} (1 - Re tr U_{mu nu}(x) / 3).

    Written with the usual plaquette U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag.
    """
    S = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Umu = U[..., mu, :, :]
            Unu = U[..., nu, :, :]
            Unu_xmu = _shift(Unu, mu, 1)
            Umu_xnu = _shift(Umu, nu, 1)
            P = Umu @ Unu_xmu @ np.conj(np.swapaxes(Umu_xnu, -1, -2)) @ np.conj(np.swapaxes(Unu, -1, -2))
            S += (1.0 - np.trace(P, axis1=-2, axis2=-1).real / 3.0).sum()
    return beta * S


def fat_links(U, c):
    """Asqtad fat links and Naik long links by spelling out every term of the asqtad matrix.

    V_{n,mu} = c_1 U_{n,mu} + c_3 (three-staples, eq. 18_6_6_4) + c_5 (five-staples,
    eq. 18_6_6_5) + c_7 (seven-staples, eq. 18_6_6_6) + c_L (Lepage, eq. 18_6_6_7);
    W_{n,mu} = c_N U_{n,mu} U_{n+mu,mu} U_{n+2mu,mu} (eq. 18_6_6_3). The transverse
    directions are enumerated with itertools, each term walked as shifted link fields.
    """
    import itertools

    c1, c3, c5, c7, cL, cN = c
    V = np.zeros_like(U)
    W = np.zeros_like(U)
    signs = (1, -1)
    for mu in range(4):
        others = [a for a in range(4) if a != mu]
        acc = c1 * U[..., mu, :, :]
        for nu in others:
            for s in signs:
                acc = acc + c3 * _walk(U, [(nu, s), (mu, 1), (nu, -s)])
                acc = acc + cL * _walk(U, [(nu, s), (nu, s), (mu, 1), (nu, -s), (nu, -s)])
        for nu, rho in itertools.permutations(others, 2):
            for s1, s2 in itertools.product(signs, signs):
                acc = acc + c5 * _walk(U, [(nu, s1), (rho, s2), (mu, 1), (rho, -s2), (nu, -s1)])
        for nu, rho, sg in itertools.permutations(others, 3):
            for s1, s2, s3 in itertools.product(signs, signs, signs):
                acc = acc + c7 * _walk(U, [(nu, s1), (rho, s2), (sg, s3), (mu, 1), (sg, -s3), (rho, -s2),
                                           (nu, -s1)])
        V[..., mu, :, :] = acc
        W[..., mu, :, :] = cN * _walk(U, [(mu, 1), (mu, 1), (mu, 1)])
    return V, W
