"""Seeded synthetic inputs for the hopping-matrix path (host, FP64, numpy).

This module only draws random fields.  It holds none of the operator's
arithmetic: no hopping term, no gamma matrices, no even-odd indexing.  Both
the CPU oracle and the HIP path consume what it returns, so it is the one
piece of code they share.

Canonical host layouts (the import format of the C-ABI):

* gauge field: ``complex128[4][V][3][3]`` -- ``U[mu, lex, a, b]`` is the
  colour matrix element ``(U_mu(x))_{ab}`` of the link leaving site ``x`` in
  direction ``mu`` (``mu = 0,1,2,3 = t,x,y,z``), ``lex = ((t*LX + x)*LY + y)*LZ + z``.
* spinor on one checkerboard: ``complex128[Vh][4][3]`` (site, spin, colour).

Random numbers come from ``numpy.random.Generator(PCG64(seed))``.  Large
fields are drawn in chunks of ``CHUNK`` links (real parts, then imaginary
parts, per chunk), so the stream -- and therefore the field -- is a fixed
function of the seed and the lattice size.  The draws are sequential; only
the per-chunk matrix work runs in a thread pool.
"""

from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

CHUNK = 1 << 20
WORKERS = max(1, min(16, os.cpu_count() or 1))

# Default seeds of the five benchmark workloads (8^4 hop, 32^3x64 Qtm/CG,
# 48^3x96 mixed precision, multi-RHS, adjoint).
SEEDS = {"hop8": 1, "qtm32": 2, "mixed48": 3, "batch": 4, "adjoint24": 5}


def volume(dims):
    T, LX, LY, LZ = (int(d) for d in dims)
    return T * LX * LY * LZ


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _complex_gauss(g: np.random.Generator, shape, scale=1.0):
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    z = np.empty(shape, dtype=np.complex128)
    z.real = re
    z.imag = im
    if scale != 1.0:
        z *= scale
    return z


def _det3(m):
    return (m[:, 0, 0] * (m[:, 1, 1] * m[:, 2, 2] - m[:, 1, 2] * m[:, 2, 1])
            - m[:, 0, 1] * (m[:, 1, 0] * m[:, 2, 2] - m[:, 1, 2] * m[:, 2, 0])
            + m[:, 0, 2] * (m[:, 1, 0] * m[:, 2, 1] - m[:, 1, 1] * m[:, 2, 0]))


def _orthonormalise_columns(z):
    """QR of a batch of 3x3 complex matrices with a positive real diagonal of
    R (Gram-Schmidt, applied twice for stability).  For complex Gaussian
    input the result is Haar-distributed on U(3) (Mezzadri's phase fix)."""
    q = z.copy()
    for _ in range(2):
        for j in range(3):
            v = q[:, :, j]
            for k in range(j):
                u = q[:, :, k]
                v -= np.einsum("ni,ni->n", u.conj(), v)[:, None] * u
            v /= np.sqrt(np.einsum("ni,ni->n", v.conj(), v).real)[:, None]
    return q


def _chunked(n, draw, work):
    """out[s:e] = work(draw(e - s)) over chunks of CHUNK, draws in order."""
    out = np.empty((n, 3, 3), dtype=np.complex128)
    with cf.ThreadPoolExecutor(WORKERS) as ex:
        pending = []
        for s in range(0, n, CHUNK):
            e = min(n, s + CHUNK)
            pending.append((s, e, ex.submit(work, draw(e - s))))
            if len(pending) >= 2 * WORKERS:
                s0, e0, f = pending.pop(0)
                out[s0:e0] = f.result()
        for s0, e0, f in pending:
            out[s0:e0] = f.result()
    return out


def _su3_from_gauss(z):
    q = _orthonormalise_columns(z)
    d = _det3(q)
    q /= (d ** (1.0 / 3.0))[:, None, None]
    return q


def haar_su3(n: int, g: np.random.Generator) -> np.ndarray:
    """``n`` Haar-random SU(3) matrices: complex Gaussian 3x3 from the
    generator, QR-orthonormalised, then divided by the principal cube root of
    the determinant so that det = 1."""
    return _chunked(n, lambda m: _complex_gauss(g, (m, 3, 3), 1.0 / np.sqrt(2.0)), _su3_from_gauss)


def gauge_haar(dims, seed: int) -> np.ndarray:
    """Haar-random gauge field, ``complex128[4][V][3][3]``."""
    V = volume(dims)
    g = rng(seed)
    return haar_su3(4 * V, g).reshape(4, V, 3, 3)


def gauge_unit(dims) -> np.ndarray:
    """Free field U = 1."""
    V = volume(dims)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices (standard normalisation tr l_a l_b = 2 delta)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def _expi(h, eps, order=12, squarings=3):
    """exp(i eps H) for H = sum_a h_a lambda_a/2: Taylor series of order 12
    on exp(i eps H / 8), squared three times (error ~1e-16 for the
    |eps H| <~ 2 drawn here; unitary with det 1 to rounding since H is
    Hermitian traceless)."""
    lam = gell_mann() / 2.0
    A = np.einsum("na,aij->nij", h, lam) * (1j * eps / 2 ** squarings)
    E = np.zeros_like(A)
    E[:, 0, 0] = E[:, 1, 1] = E[:, 2, 2] = 1.0
    term = E.copy()
    for k in range(1, order + 1):
        term = np.einsum("nij,njk->nik", term, A) / k
        E += term
    for _ in range(squarings):
        E = np.einsum("nij,njk->nik", E, E)
    return E


def gauge_smooth(dims, seed: int, eps: float) -> np.ndarray:
    """Links smoothed toward the identity: ``U = exp(i eps H)`` with
    ``H = sum_a h_a lambda_a / 2``, ``h_a ~ N(0,1)`` (Gaussian Hermitian
    traceless)."""
    V = volume(dims)
    g = rng(seed)
    out = _chunked(4 * V, lambda m: g.standard_normal((m, 8)), lambda h: _expi(h, eps))
    return out.reshape(4, V, 3, 3)


def gauge_transform(dims, seed: int) -> np.ndarray:
    """A random site-wise SU(3) gauge transformation ``Omega[lex]``."""
    return haar_su3(volume(dims), rng(seed))


def spinor_gauss(nsites: int, seed: int) -> np.ndarray:
    """Complex Gaussian spinor ``complex128[nsites][4][3]``; real and imaginary
    parts are independent N(0,1)."""
    g = rng(seed)
    n = int(nsites) * 12
    out = np.empty(n, dtype=np.complex128)
    for s in range(0, n, 12 * CHUNK):
        e = min(n, s + 12 * CHUNK)
        out[s:e] = _complex_gauss(g, (e - s,))
    return out.reshape(int(nsites), 4, 3)
