"""Pins of the CPU oracle against facts that do not come from the oracle.

* closed forms: the free-field (U = 1) plane-wave symbol of the hopping term
  and the free-field eigenvalue of Qhat^dagger Qhat (derived at
  ``free_lambda``);
* invariants: gauge covariance under random SU(3) transformations,
  gamma_5-hermiticity of the hopping term, Qhat(+)^dagger = Qhat(-);
* brute force: dense matrices built independently in ``tests/dense.py`` on
  2^4 and 6x2x4x2 lattices, the Schur complement through numpy.linalg.inv,
  the determinant identity log det M = log det M_ee + log det Mhat, and CG
  against numpy.linalg.solve;
* the Clifford algebra of the gamma matrices and the even-odd site order.
"""

import numpy as np
import pytest

import fieldgen
import oracle
import dense


def plane_wave(dims, parity, n, theta, u):
    """psi(x) = exp(i p.x) u on the sites of one parity, even-odd order, with
    p_mu = (2 n_mu + theta_mu) pi / L_mu (satisfies the twisted boundary)."""
    c = dense.coords(dims)[dense.parity_sites(dims, parity)]
    p = np.array([(2 * n[m] + theta[m]) * np.pi / dims[m] for m in range(4)])
    ph = np.exp(1j * (c @ p))
    return ph[:, None, None] * u[None, :, :], p, ph


def free_symbol(p, kappa):
    """kappa (2 sum_mu cos p_mu - 2 i sum_mu gamma_mu sin p_mu), 4x4."""
    g, _ = dense.gammas()
    return kappa * (2 * np.sum(np.cos(p)) * np.eye(4)
                    - 2j * sum(np.sin(p[m]) * g[m] for m in range(4)))


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ----------------------------------------------------------------- gammas

def test_gamma_clifford_and_basis():
    g = [oracle.gamma(m) for m in range(4)]
    g5 = oracle.gamma(4)
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T, atol=0)
        for n in range(4):
            ac = g[m] @ g[n] + g[n] @ g[m]
            assert np.allclose(ac, 2 * np.eye(4) * (m == n), atol=0)
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=0)
    gd, g5d = dense.gammas()
    for m in range(4):
        assert np.array_equal(g[m], gd[m])
    assert np.array_equal(g5, g5d)


def test_even_odd_order_is_lex_half():
    """The k-th site of parity p in lex order is lex = 2k or 2k+1 (LZ even):
    the even-odd index is lex >> 1."""
    for dims in [(2, 2, 2, 2), (6, 2, 4, 2), (4, 6, 8, 2), (8, 4, 4, 6)]:
        for p in (0, 1):
            lex = oracle.eo_sites(dims, p)
            assert np.array_equal(lex, dense.parity_sites(dims, p))
            assert np.array_equal(lex >> 1, np.arange(len(lex)))


# ------------------------------------------------------- free-field symbol

@pytest.mark.parametrize("dims,theta", [
    ((4, 6, 2, 8), (1.0, 0.0, 0.0, 0.0)),
    ((8, 4, 4, 4), (1.0, 0.0, 0.0, 0.0)),
    ((6, 4, 8, 2), (0.5, 0.25, -0.3, 0.7)),
])
def test_free_field_plane_wave_hop(dims, theta):
    kappa = 0.137
    U = fieldgen.gauge_unit(dims)
    g = fieldgen.rng(11)
    for n in [(0, 0, 0, 0), (1, 2, 0, 3), (3, 1, 1, 0), (-1, 2, 1, -2)]:
        u = g.standard_normal((4, 3)) + 1j * g.standard_normal((4, 3))
        for direction, pin, pout in (("eo", 1, 0), ("oe", 0, 1)):
            psi, p, _ = plane_wave(dims, pin, n, theta, u)
            _, _, ph_out = plane_wave(dims, pout, n, theta, u)
            out = oracle.hop(dims, direction, U, psi, kappa, theta)
            expect = ph_out[:, None, None] * (free_symbol(p, kappa) @ u)[None]
            assert rel(out, expect) < 1e-13, (direction, n)


def test_free_field_full_lattice_hop():
    dims, theta, kappa = (4, 2, 6, 4), (1.0, 0.0, 0.5, 0.0), 0.21
    U = fieldgen.gauge_unit(dims)
    u = np.arange(12).reshape(4, 3) * (1 + 0.5j) - 3
    c = dense.coords(dims)
    n = (1, 0, 2, 3)
    p = np.array([(2 * n[m] + theta[m]) * np.pi / dims[m] for m in range(4)])
    ph = np.exp(1j * (c @ p))
    psi = ph[:, None, None] * u[None]
    out = oracle.hop_full(dims, U, psi, kappa, theta)
    assert rel(out, ph[:, None, None] * (free_symbol(p, kappa) @ u)[None]) < 1e-13


def test_constant_field_special_case():
    """U = 1, theta = 0, psi = const u  ->  H psi = 8 kappa u."""
    dims, kappa = (4, 4, 2, 6), 0.16
    U = fieldgen.gauge_unit(dims)
    u = (np.arange(12) + 1j).reshape(4, 3)
    psi = np.broadcast_to(u, (np.prod(dims) // 2, 4, 3)).copy()
    for d in ("eo", "oe"):
        out = oracle.hop(dims, d, U, psi, kappa, (0, 0, 0, 0))
        assert np.allclose(out, 8 * kappa * u[None], rtol=1e-15, atol=1e-14)


# ------------------------------------------------------------- invariants

def gauge_rotate(dims, U, Om):
    """U^Om_mu(x) = Om(x) U_mu(x) Om(x+mu)^dagger."""
    c = dense.coords(dims)
    out = np.empty_like(U)
    for mu in range(4):
        cf = c.copy()
        cf[:, mu] = (cf[:, mu] + 1) % dims[mu]
        nb = np.ravel_multi_index(tuple(cf.T), dims)
        out[mu] = Om @ U[mu] @ Om[nb].conj().transpose(0, 2, 1)
    return out


@pytest.mark.parametrize("dims", [(4, 6, 2, 4), (2, 2, 2, 2), (6, 4, 4, 8)])
def test_gauge_covariance(dims):
    theta, kappa, mu = (1.0, 0.0, 0.0, 0.0), 0.15, 0.05
    U = fieldgen.gauge_haar(dims, 21)
    Om = fieldgen.gauge_transform(dims, 22)
    UO = gauge_rotate(dims, U, Om)
    Vh = np.prod(dims) // 2
    ev, od = dense.parity_sites(dims, 0), dense.parity_sites(dims, 1)
    for direction, pin, sin_, sout in (("eo", 1, od, ev), ("oe", 0, ev, od)):
        psi = fieldgen.spinor_gauss(Vh, 23 + pin)
        psiO = np.einsum("nab,nsb->nsa", Om[sin_], psi)
        lhs = oracle.hop(dims, direction, UO, psiO, kappa, theta)
        rhs = np.einsum("nab,nsb->nsa", Om[sout], oracle.hop(dims, direction, U, psi, kappa, theta))
        assert rel(lhs, rhs) < 1e-13
    psi = fieldgen.spinor_gauss(Vh, 25)
    psiO = np.einsum("nab,nsb->nsa", Om[od], psi)
    lhs = oracle.qtm(dims, UO, psiO, kappa, mu, theta, +1)
    rhs = np.einsum("nab,nsb->nsa", Om[od], oracle.qtm(dims, U, psi, kappa, mu, theta, +1))
    assert rel(lhs, rhs) < 1e-13


def test_gauge_covariance_detects_transposed_link():
    """The covariance pin is not vacuous: U^T in place of U breaks it."""
    dims, theta, kappa = (4, 2, 4, 2), (1.0, 0, 0, 0), 0.15
    U = fieldgen.gauge_haar(dims, 31)
    Om = fieldgen.gauge_transform(dims, 32)
    UT = U.transpose(0, 1, 3, 2).copy()
    UTO = gauge_rotate(dims, U, Om).transpose(0, 1, 3, 2).copy()
    psi = fieldgen.spinor_gauss(np.prod(dims) // 2, 33)
    od, ev = dense.parity_sites(dims, 1), dense.parity_sites(dims, 0)
    psiO = np.einsum("nab,nsb->nsa", Om[od], psi)
    lhs = oracle.hop(dims, "eo", UTO, psiO, kappa, theta)
    rhs = np.einsum("nab,nsb->nsa", Om[ev], oracle.hop(dims, "eo", UT, psi, kappa, theta))
    assert rel(lhs, rhs) > 1e-2


def g5(psi):
    out = psi.copy()
    out[:, 2:, :] *= -1
    return out


@pytest.mark.parametrize("dims", [(4, 6, 2, 4), (8, 4, 4, 2)])
def test_gamma5_hermiticity(dims):
    """<chi_e, H_eo psi_o> = <gamma_5 H_oe gamma_5 chi_e, psi_o>."""
    theta, kappa = (1.0, 0.3, 0.0, -0.5), 0.16
    U = fieldgen.gauge_haar(dims, 41)
    Vh = np.prod(dims) // 2
    chi = fieldgen.spinor_gauss(Vh, 42)
    psi = fieldgen.spinor_gauss(Vh, 43)
    lhs = np.vdot(chi, oracle.hop(dims, "eo", U, psi, kappa, theta))
    rhs = np.vdot(g5(oracle.hop(dims, "oe", U, g5(chi), kappa, theta)), psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs) + 1e-12


def test_qtm_plus_dagger_is_qtm_minus():
    dims, theta, kappa, mu = (4, 4, 2, 6), (1.0, 0, 0, 0), 0.1632, 0.0013 / (2 * 0.1632)
    U = fieldgen.gauge_haar(dims, 51)
    Vh = np.prod(dims) // 2
    chi = fieldgen.spinor_gauss(Vh, 52)
    psi = fieldgen.spinor_gauss(Vh, 53)
    lhs = np.vdot(chi, oracle.qtm(dims, U, psi, kappa, mu, theta, +1))
    rhs = np.vdot(oracle.qtm(dims, U, chi, kappa, mu, theta, -1), psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


# ------------------------------------------------------------ brute force

@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (6, 2, 4, 2)])
def test_hop_matches_dense(dims):
    theta, kappa = (1.0, 0.0, 0.5, 0.0), 0.16
    U = fieldgen.gauge_haar(dims, 61)
    V = int(np.prod(dims))
    H = dense.hopping_matrix(dims, U, kappa, theta)
    ee, eo, oe, oo = dense.eo_blocks(dims, H)
    assert np.abs(ee).max() == 0 and np.abs(oo).max() == 0
    for direction, blk, seed in (("eo", eo, 62), ("oe", oe, 63)):
        psi = fieldgen.spinor_gauss(V // 2, seed)
        out = oracle.hop(dims, direction, U, psi, kappa, theta)
        assert rel(out.ravel(), blk @ psi.ravel()) < 1e-14
    psi = fieldgen.spinor_gauss(V, 64)
    assert rel(oracle.hop_full(dims, U, psi, kappa, theta).ravel(), H @ psi.ravel()) < 1e-14


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (6, 2, 4, 2)])
def test_qtm_matches_dense_schur(dims):
    theta, kappa, mu = (1.0, 0.0, 0.0, 0.0), 0.16, 0.37
    U = fieldgen.gauge_haar(dims, 71)
    Vh = int(np.prod(dims)) // 2
    psi = fieldgen.spinor_gauss(Vh, 72)
    for sign in (+1, -1):
        Q, M, Mhat = dense.schur_qhat(dims, U, kappa, mu, theta, sign)
        out = oracle.qtm(dims, U, psi, kappa, mu, theta, sign)
        assert rel(out.ravel(), Q @ psi.ravel()) < 1e-13
        if sign == +1:
            Qp = Q
        else:
            assert np.allclose(Qp.conj().T, Q, atol=1e-13)
    # log det M = log det M_ee + log det Mhat (Schur complement)
    _, M, Mhat = dense.schur_qhat(dims, U, kappa, mu, theta, +1)
    ee, _, _, _ = dense.eo_blocks(dims, M)
    s_full, l_full = np.linalg.slogdet(M)
    s_ee, l_ee = np.linalg.slogdet(ee)
    s_h, l_h = np.linalg.slogdet(Mhat)
    assert abs(l_full - (l_ee + l_h)) < 1e-12 * abs(l_full) + 1e-11
    assert abs(s_full - s_ee * s_h) < 1e-10


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (6, 2, 4, 2)])
def test_full_operator_matches_dense(dims):
    theta, kappa, mu = (1.0, 0.0, 0.5, 0.0), 0.16, 0.37
    U = fieldgen.gauge_haar(dims, 75)
    psi = fieldgen.spinor_gauss(int(np.prod(dims)), 76)
    for sign in (+1, -1):
        M = dense.full_operator(dims, U, kappa, mu, theta, sign)
        out = oracle.full_operator(dims, U, psi, kappa, mu, theta, sign)
        assert rel(out.ravel(), M @ psi.ravel()) < 1e-14


def test_cg_matches_dense_solve():
    dims, theta, kappa, mu = (2, 2, 2, 2), (1.0, 0, 0, 0), 0.1632, 0.0013 / (2 * 0.1632)
    U = fieldgen.gauge_haar(dims, 81)
    Vh = int(np.prod(dims)) // 2
    b = fieldgen.spinor_gauss(Vh, 82)
    Q, _, _ = dense.schur_qhat(dims, U, kappa, mu, theta, +1)
    A = Q.conj().T @ Q
    x_ref = np.linalg.solve(A, b.ravel())
    x, it, res, ok = oracle.cg(dims, U, b, kappa, mu, theta, tol=1e-12)
    assert ok and res <= 1e-12
    assert rel(x.ravel(), x_ref) < 1e-12 * np.linalg.cond(A)


# ------------------------------------------------------- free-field Qtm/CG

def free_lambda(p, kappa, mt):
    """Eigenvalue of Mhat^dagger Mhat on a free plane wave of momentum p.

    On the wave both hops act as K = a - i B with a = 2 kappa sum cos p_mu
    and B = 2 kappa sum gamma_mu sin p_mu, B^2 = s2 = 4 kappa^2 sum sin^2 p_mu.
    With A = 1 + i mt gamma_5, A^-1 = (1 - i mt gamma_5) / D, D = 1 + mt^2,
    and gamma_5 B = -B gamma_5:
    K A^-1 K = [(a^2 - s2) - 2 i a B - i mt (a^2 + s2) gamma_5] / D, so
    Mhat = A - K A^-1 K = alpha + i beta gamma_5 + i (2a / D) B with the
    alpha, beta below; in Mhat^dagger Mhat the cross terms in
    gamma_5 B + B gamma_5 vanish, leaving alpha^2 + beta^2 + (2a / D)^2 s2."""
    a = 2 * kappa * np.sum(np.cos(p))
    s2 = 4 * kappa ** 2 * np.sum(np.sin(p) ** 2)
    D = 1 + mt ** 2
    alpha = (D - a * a + s2) / D
    beta = mt * (D + a * a + s2) / D
    return alpha ** 2 + beta ** 2 + 4 * a * a * s2 / D ** 2


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 0, 3), (2, 0, 1, 1)])
def test_free_field_normal_operator_eigenvalue(n):
    dims, theta, kappa, mu = (8, 4, 4, 6), (1.0, 0, 0, 0), 0.1632, 0.05
    U = fieldgen.gauge_unit(dims)
    u = fieldgen.rng(91).standard_normal((4, 3)) + 0j
    psi, p, _ = plane_wave(dims, 1, n, theta, u)
    lam = free_lambda(p, kappa, 2 * kappa * mu)
    out = oracle.normal(dims, U, psi, kappa, mu, theta)
    assert rel(out, lam * psi) < 1e-13


def test_cg_free_plane_wave_one_iteration():
    dims, theta, kappa, mu = (8, 4, 4, 6), (1.0, 0, 0, 0), 0.1632, 0.0013 / (2 * 0.1632)
    U = fieldgen.gauge_unit(dims)
    u = fieldgen.rng(92).standard_normal((4, 3)) + 1j
    b, p, _ = plane_wave(dims, 1, (1, 0, 2, 1), theta, u)
    lam = free_lambda(p, kappa, 2 * kappa * mu)
    x, it, res, ok = oracle.cg(dims, U, b, kappa, mu, theta, tol=1e-12)
    assert ok and it == 1
    assert rel(x, b / lam) < 1e-12


def test_cg_random_converges_true_residual():
    dims, theta, kappa, mu = (4, 4, 4, 4), (1.0, 0, 0, 0), 0.1632, 0.0013 / (2 * 0.1632)
    U = fieldgen.gauge_haar(dims, 93)
    b = fieldgen.spinor_gauss(np.prod(dims) // 2, 94)
    x, it, res, ok = oracle.cg(dims, U, b, kappa, mu, theta, tol=1e-10)
    assert ok and res <= 1e-10 and it > 5
    r = b - oracle.normal(dims, U, x, kappa, mu, theta)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10


def test_cg_not_converged_reports():
    dims, theta, kappa, mu = (4, 4, 4, 4), (1.0, 0, 0, 0), 0.1632, 0.0013 / (2 * 0.1632)
    U = fieldgen.gauge_haar(dims, 95)
    b = fieldgen.spinor_gauss(np.prod(dims) // 2, 96)
    x, it, res, ok = oracle.cg(dims, U, b, kappa, mu, theta, tol=1e-10, max_iter=2)
    assert not ok and it == 2 and res > 1e-10


# ------------------------------------------------------------- generators

def test_haar_su3_properties():
    g = fieldgen.rng(101)
    Us = fieldgen.haar_su3(200000, g)
    eye = np.eye(3)
    assert np.abs(Us @ Us.conj().transpose(0, 2, 1) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(Us) - 1).max() < 1e-14
    # Haar moments: E|U_ab|^2 = 1/3, E U_ab = 0
    m2 = np.mean(np.abs(Us) ** 2, axis=0)
    assert np.abs(m2 - 1 / 3).max() < 5e-3
    assert np.abs(Us.mean(axis=0)).max() < 5e-3


def test_smooth_links_properties():
    dims = (2, 2, 2, 4)
    U = fieldgen.gauge_smooth(dims, 102, 0.3).reshape(-1, 3, 3)
    assert np.abs(U @ U.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    assert np.abs(np.trace(U, axis1=1, axis2=2).real / 3 - 1).mean() < 0.1


def test_generators_are_deterministic():
    a = fieldgen.gauge_haar((2, 2, 2, 2), 7)
    b = fieldgen.gauge_haar((2, 2, 2, 2), 7)
    assert np.array_equal(a, b)
    assert np.array_equal(fieldgen.spinor_gauss(10, 3), fieldgen.spinor_gauss(10, 3))


def test_thread_count_does_not_change_results():
    """Each output site is computed by one thread from the inputs alone, so
    the hop is bitwise the same on one thread and on all of them."""
    dims = (4, 6, 2, 6)
    U = fieldgen.gauge_haar(dims, 61)
    psi = fieldgen.spinor_gauss(int(np.prod(dims)) // 2, 62)
    n = oracle.num_threads()
    try:
        oracle.set_num_threads(1)
        assert oracle.num_threads() == 1
        one = oracle.hop(dims, "eo", U, psi, 0.16, (1.0, 0.3, 0.0, 0.0))
    finally:
        oracle.set_num_threads(n)
    assert oracle.num_threads() == n
    many = oracle.hop(dims, "eo", U, psi, 0.16, (1.0, 0.3, 0.0, 0.0))
    assert np.array_equal(one, many)
