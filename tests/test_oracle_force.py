"""Pins of the oracle's gauge-link derivative (force) against central finite
differences of the oracle's own, already pinned, operators.

A link U_mu(l) is moved along exp(+-h T) with T = i lambda_a / 2 (a basis of
su(3)) and the change of L is compared with tr(T F), F = the su(3) force.
The difference L(+h) - L(-h) is formed from the site-wise difference of the
two operator applications: sites the link cannot reach give bitwise-equal
values, so only the terms within two hops of the link contribute and the
roundoff of the full sum never enters (step 1e-6, agreement 1e-6 per link
over the 8 components).
"""

import numpy as np
import pytest

import fieldgen
import oracle

H_STEP = 1e-6
LAM = fieldgen.gell_mann()
GEN = 1j * LAM / 2          # anti-Hermitian traceless basis of su(3)


def expm_herm(A):
    """exp(i A) for Hermitian A (numpy eigh)."""
    w, v = np.linalg.eigh(A)
    return (v * np.exp(1j * w)) @ v.conj().T


def kahan_re_dot(a, b):
    return oracle.re_dot(np.ascontiguousarray(a), np.ascontiguousarray(b))


def perturbed(U, mu, l, a, h):
    Up = U.copy()
    Up[mu, l] = expm_herm(h * LAM[a] / 2) @ U[mu, l]
    return Up


def check_links(dims, U, F, dL, links, rtol=1e-6):
    worst = 0.0
    for mu, l in links:
        fd = np.array([dL(mu, l, a) for a in range(8)])
        an = np.array([np.trace(GEN[a] @ F[mu, l]).real for a in range(8)])
        err = np.linalg.norm(fd - an) / np.linalg.norm(an)
        worst = max(worst, err)
        assert err < rtol, (mu, l, err, fd, an)
    return worst


def sample_links(dims, n, seed):
    g = fieldgen.rng(seed)
    V = int(np.prod(dims))
    return [(int(g.integers(0, 4)), int(g.integers(0, V))) for _ in range(n)]


@pytest.mark.parametrize("direction", ["eo", "oe"])
@pytest.mark.parametrize("dims,theta", [((4, 2, 4, 6), (1.0, 0, 0, 0)),
                                        ((2, 4, 2, 4), (0.5, 0.3, 0.0, -0.7))])
def test_hop_force_finite_differences(dims, theta, direction):
    kappa = 0.15
    U = fieldgen.gauge_haar(dims, 201)
    Vh = int(np.prod(dims)) // 2
    X, Y = fieldgen.spinor_gauss(Vh, 202), fieldgen.spinor_gauss(Vh, 203)
    F = oracle.hop_force(dims, direction, U, X, Y, kappa, theta)

    def dL(mu, l, a):
        hp = oracle.hop(dims, direction, perturbed(U, mu, l, a, H_STEP), Y, kappa, theta)
        hm = oracle.hop(dims, direction, perturbed(U, mu, l, a, -H_STEP), Y, kappa, theta)
        return kahan_re_dot(X, hp - hm) / (2 * H_STEP)

    # every link of a 2x4x2x4 lattice, a sample of the larger one
    V = int(np.prod(dims))
    links = [(m, l) for m in range(4) for l in range(V)] if V <= 64 else sample_links(dims, 48, 204)
    check_links(dims, U, F, dL, links)


def test_force_is_su3():
    dims, theta = (4, 2, 4, 6), (1.0, 0, 0, 0)
    U = fieldgen.gauge_haar(dims, 211)
    Vh = int(np.prod(dims)) // 2
    F = oracle.qtm_force(dims, U, fieldgen.spinor_gauss(Vh, 212), fieldgen.spinor_gauss(Vh, 213),
                         0.16, 0.2, theta)
    Fd = F.conj().transpose(0, 1, 3, 2)
    assert np.abs(F + Fd).max() < 1e-14
    assert np.abs(np.trace(F, axis1=2, axis2=3)).max() < 1e-14
    assert np.abs(F).max() > 1e-3


@pytest.mark.parametrize("sign", [+1, -1])
def test_qtm_force_finite_differences(sign):
    dims, theta, kappa, mu = (4, 2, 4, 6), (1.0, 0, 0, 0), 0.16, 0.6
    U = fieldgen.gauge_haar(dims, 221)
    Vh = int(np.prod(dims)) // 2
    chi, psi = fieldgen.spinor_gauss(Vh, 222), fieldgen.spinor_gauss(Vh, 223)
    F = oracle.qtm_force(dims, U, chi, psi, kappa, mu, theta, sign)

    def dL(m, l, a):
        qp = oracle.qtm(dims, perturbed(U, m, l, a, H_STEP), psi, kappa, mu, theta, sign)
        qm = oracle.qtm(dims, perturbed(U, m, l, a, -H_STEP), psi, kappa, mu, theta, sign)
        return kahan_re_dot(chi, qp - qm) / (2 * H_STEP)

    check_links(dims, U, F, dL, sample_links(dims, 40, 224))


def test_qtm_norm_force_finite_differences():
    """L = |Qhat psi|^2 has force qtm_force(chi = 2 Qhat psi); the difference
    |a|^2 - |b|^2 is formed as Re <a - b, a + b>."""
    dims, theta, kappa, mu = (2, 4, 2, 4), (1.0, 0, 0, 0), 0.16, 0.3
    U = fieldgen.gauge_haar(dims, 231)
    Vh = int(np.prod(dims)) // 2
    psi = fieldgen.spinor_gauss(Vh, 232)
    chi = 2 * oracle.qtm(dims, U, psi, kappa, mu, theta, +1)
    F = oracle.qtm_force(dims, U, chi, psi, kappa, mu, theta, +1)

    def dL(m, l, a):
        qp = oracle.qtm(dims, perturbed(U, m, l, a, H_STEP), psi, kappa, mu, theta, +1)
        qm = oracle.qtm(dims, perturbed(U, m, l, a, -H_STEP), psi, kappa, mu, theta, +1)
        return kahan_re_dot(qp - qm, qp + qm) / (2 * H_STEP)

    V = int(np.prod(dims))
    check_links(dims, U, F, dL, [(m, l) for m in range(4) for l in range(V)])


def test_euclidean_gradient_finite_differences():
    """kind='euclid': dL = Re sum conj(G) dU for any complex dU (no SU(3)
    constraint); checked along random complex directions per link."""
    dims, theta, kappa, mu = (2, 4, 2, 4), (0.5, 0, 0, 0), 0.16, 0.3
    U = fieldgen.gauge_haar(dims, 241)
    Vh = int(np.prod(dims)) // 2
    chi, psi = fieldgen.spinor_gauss(Vh, 242), fieldgen.spinor_gauss(Vh, 243)
    G = oracle.qtm_force(dims, U, chi, psi, kappa, mu, theta, -1, kind="euclid")
    g = fieldgen.rng(244)
    for mu_, l in sample_links(dims, 24, 245):
        E = g.standard_normal((3, 3)) + 1j * g.standard_normal((3, 3))
        Up, Um = U.copy(), U.copy()
        Up[mu_, l] += H_STEP * E
        Um[mu_, l] -= H_STEP * E
        qp = oracle.qtm(dims, Up, psi, kappa, mu, theta, -1)
        qm = oracle.qtm(dims, Um, psi, kappa, mu, theta, -1)
        fd = kahan_re_dot(chi, qp - qm) / (2 * H_STEP)
        an = np.sum(G[mu_, l].conj() * E).real
        assert abs(fd - an) <= 1e-7 * (abs(an) + np.abs(G[mu_, l]).sum())


def test_force_kinds_agree():
    """For the left variation U -> exp(tZ) U the Euclidean gradient G gives
    dL/dt = Re tr(Z U G^+), so TA(U G^+) must equal the su(3) force."""
    dims, theta = (2, 4, 2, 4), (1.0, 0, 0, 0)
    U = fieldgen.gauge_haar(dims, 251)
    Vh = int(np.prod(dims)) // 2
    X, Y = fieldgen.spinor_gauss(Vh, 252), fieldgen.spinor_gauss(Vh, 253)
    F = oracle.hop_force(dims, "oe", U, X, Y, 0.2, theta)
    G = oracle.hop_force(dims, "oe", U, X, Y, 0.2, theta, kind="euclid")
    M = U @ G.conj().transpose(0, 1, 3, 2)
    A = (M - M.conj().transpose(0, 1, 3, 2)) / 2
    TA = A - np.einsum("mlii->ml", A)[:, :, None, None] * np.eye(3) / 3
    assert np.abs(TA - F).max() < 1e-14


def test_force_detects_wrong_sign():
    """The finite-difference pin is not vacuous: the negated force fails it."""
    dims, theta, kappa = (2, 4, 2, 4), (1.0, 0, 0, 0), 0.15
    U = fieldgen.gauge_haar(dims, 261)
    Vh = int(np.prod(dims)) // 2
    X, Y = fieldgen.spinor_gauss(Vh, 262), fieldgen.spinor_gauss(Vh, 263)
    F = -oracle.hop_force(dims, "eo", U, X, Y, kappa, theta)

    def dL(mu, l, a):
        hp = oracle.hop(dims, "eo", perturbed(U, mu, l, a, H_STEP), Y, kappa, theta)
        hm = oracle.hop(dims, "eo", perturbed(U, mu, l, a, -H_STEP), Y, kappa, theta)
        return kahan_re_dot(X, hp - hm) / (2 * H_STEP)

    with pytest.raises(AssertionError):
        check_links(dims, U, F, dL, sample_links(dims, 4, 264))
