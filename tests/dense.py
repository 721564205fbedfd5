"""Brute-force dense matrices for tiny lattices (numpy), used to pin the oracle.

Everything here is built independently of ``oracle/``: the gamma matrices
come from the Pauli matrices, sites are walked in lexicographic order with
numpy's ``unravel_index``, the hopping term is assembled block by block as
``kron(spin matrix, colour matrix)`` into a dense ``12V x 12V`` matrix, and
the even-odd Schur complement is formed with ``numpy.linalg.inv``.

Row/column index of a full-lattice spinor entry: ``(lex*4 + spin)*3 + colour``.
"""

from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
SIGMA = [np.array([[0, 1], [1, 0]], dtype=np.complex128),
         np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
         np.array([[1, 0], [0, -1]], dtype=np.complex128)]


def gammas():
    """Chiral basis: gamma_mu = [[0, e_mu], [e_mu^+, 0]] with e_0 = -1 and
    e_k = -i sigma_k; gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3."""
    e = [-I2] + [-1j * s for s in SIGMA]
    Z = np.zeros((2, 2), dtype=np.complex128)
    g = [np.block([[Z, em], [em.conj().T, Z]]) for em in e]
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


def coords(dims):
    """Coordinates (t, x, y, z) of every site in lex order, shape [V, 4]."""
    V = int(np.prod(dims))
    return np.stack(np.unravel_index(np.arange(V), tuple(dims)), axis=1)


def parity_sites(dims, p):
    """Lex indices of the sites of parity p, in lex order (= even-odd order)."""
    c = coords(dims)
    return np.nonzero(c.sum(axis=1) % 2 == p)[0]


def hopping_matrix(dims, U, kappa, theta):
    """Dense full-lattice hopping term H (kappa included)."""
    dims = tuple(int(d) for d in dims)
    V = int(np.prod(dims))
    g, _ = gammas()
    one = np.eye(4, dtype=np.complex128)
    H = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    c = coords(dims)
    for x in range(V):
        for mu in range(4):
            cf = c[x].copy()
            cf[mu] = (cf[mu] + 1) % dims[mu]
            yf = int(np.ravel_multi_index(tuple(cf), dims))
            eta_f = np.exp(1j * np.pi * theta[mu]) if c[x][mu] == dims[mu] - 1 else 1.0
            cb = c[x].copy()
            cb[mu] = (cb[mu] - 1) % dims[mu]
            yb = int(np.ravel_multi_index(tuple(cb), dims))
            eta_b = np.exp(-1j * np.pi * theta[mu]) if c[x][mu] == 0 else 1.0
            H[12 * x:12 * x + 12, 12 * yf:12 * yf + 12] += \
                kappa * eta_f * np.kron(one - g[mu], U[mu, x])
            H[12 * x:12 * x + 12, 12 * yb:12 * yb + 12] += \
                kappa * eta_b * np.kron(one + g[mu], U[mu, yb].conj().T)
    return H


def eo_blocks(dims, M):
    """Split a full-lattice matrix into (ee, eo, oe, oo) blocks, even-odd order."""
    ev = parity_sites(dims, 0)
    od = parity_sites(dims, 1)
    ie = (12 * ev[:, None] + np.arange(12)[None, :]).ravel()
    io = (12 * od[:, None] + np.arange(12)[None, :]).ravel()
    return M[np.ix_(ie, ie)], M[np.ix_(ie, io)], M[np.ix_(io, ie)], M[np.ix_(io, io)]


def twist(nsites, mt):
    """Site-diagonal 1 + i mt gamma_5 on nsites sites."""
    _, g5 = gammas()
    return np.kron(np.eye(nsites), np.kron(np.eye(4) + 1j * mt * g5, np.eye(3)))


def gamma5_field(nsites):
    _, g5 = gammas()
    return np.kron(np.eye(nsites), np.kron(g5, np.eye(3)))


def full_operator(dims, U, kappa, mu, theta, sign=+1):
    """M = (1 + i s 2 kappa mu gamma_5) - H on the full lattice."""
    V = int(np.prod(dims))
    H = hopping_matrix(dims, U, kappa, theta)
    return twist(V, sign * 2 * kappa * mu) - H


def schur_qhat(dims, U, kappa, mu, theta, sign=+1):
    """Qhat = gamma_5 (M_oo - M_oe M_ee^-1 M_eo), via numpy.linalg.inv."""
    M = full_operator(dims, U, kappa, mu, theta, sign)
    ee, eo, oe, oo = eo_blocks(dims, M)
    Mhat = oo - oe @ np.linalg.inv(ee) @ eo
    return gamma5_field(ee.shape[0] // 12) @ Mhat, M, Mhat
