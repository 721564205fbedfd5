"""FP16 storage (TMH_F16, TMH_F16_R12: binary16 words, FP32 arithmetic) on
the GPU against the oracle.

The oracle is fed the same FP16-rounded inputs the GPU reads (for two-row
links: the rounded first two rows and the third rebuilt from them), so what
is left is the kernel's own error: FP32 arithmetic (~1e-6) and the rounding
of every stored result to FP16, at most 2^-11 relative per component.  The
bars follow from that: 2^-11 per site for one hop (its output is rounded
once) and 3 * 2^-11 for Qtm (the even intermediate is rounded too, and its
error passes through a second hop).  The solver with an FP16 inner code must
still reach 1e-10 under the oracle's FP64 operator."""

import numpy as np
import pytest

import fieldgen
import oracle
import paper_1311_4521_amd as tm
from paper_1311_4521_amd import tmhop
from helpers import QTM32, THETA_AP, gauss, haar, mu_of, site_rel_err

pytestmark = pytest.mark.gpu

F16S = [tm.F16, tm.F16_R12]
PID = {tm.F16: "f16", tm.F16_R12: "f16r12"}
HOP_TOL = 2.0 ** -11 + 2e-6
QTM_TOL = 3 * 2.0 ** -11
SMALL = [(2, 2, 2, 2), (6, 2, 4, 2), (4, 6, 2, 6), (6, 8, 10, 4), (8, 6, 4, 10)]
THETAS = [THETA_AP, (0.5, 0.25, -0.3, 0.7)]


def to_host(t):
    return t.detach().cpu().numpy()


def round_f16(a):
    """FP64 -> FP16 (one rounding to nearest even) -> FP64, component-wise:
    what import stores."""
    a = np.asarray(a)
    f = lambda x: x.astype(np.float16).astype(np.float64)
    return f(a.real) + 1j * f(a.imag)


def links_seen(U, prec):
    """The links the kernel multiplies with: rounded entries, and for two-row
    storage the third row rebuilt from the rounded first two."""
    Uh = round_f16(U)
    if prec == tm.F16_R12:
        Uh = Uh.copy()
        Uh[..., 2, :] = np.conj(np.cross(Uh[..., 0, :], Uh[..., 1, :]))
    return Uh


def run_hop(dims, U, psi, direction, kappa, theta, prec):
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U, prec)
    x = tm.spinor_import(lat, psi, prec)
    out = lat.new_spinor(prec)
    tm.hop_apply(lat, direction, out, G, x, kappa, theta, prec)
    return to_host(tm.spinor_export(lat, out, prec))


def test_roundtrip():
    dims = (4, 6, 2, 6)
    U = haar(dims, 801)
    lat = tm.Lattice(dims)
    psi = gauss(lat.Vh, 802)
    assert lat.spinor_bytes(tm.F16) * 4 == lat.spinor_bytes(tm.F64)
    assert lat.gauge_bytes(tm.F16_R12) * 3 == lat.gauge_bytes(tm.F16) * 2
    back = to_host(tm.spinor_export(lat, tm.spinor_import(lat, psi, tm.F16), tm.F16))
    want = round_f16(psi)
    bad = np.flatnonzero((back != want).ravel())
    assert bad.size == 0, [(psi.ravel()[k], back.ravel()[k], want.ravel()[k]) for k in bad[:8]]
    for prec in F16S:
        G = tm.gauge_import(lat, U, prec)
        got = to_host(tm.gauge_export(lat, G, prec))
        assert np.abs(got - links_seen(U, prec)).max() <= 1e-15


@pytest.mark.parametrize("prec", F16S, ids=PID.get)
@pytest.mark.parametrize("theta", THETAS, ids=["ap", "twisted"])
@pytest.mark.parametrize("dims", SMALL, ids=lambda d: "x".join(map(str, d)))
def test_hop_small_lattices(dims, theta, prec):
    kappa = 0.137
    U = haar(dims, 7)
    for direction, seed in (("eo", 8), ("oe", 9)):
        psi = gauss(np.prod(dims) // 2, seed)
        ref = oracle.hop(dims, direction, links_seen(U, prec), round_f16(psi), kappa, theta)
        got = run_hop(dims, U, psi, direction, kappa, theta, prec)
        assert site_rel_err(got, ref) <= HOP_TOL, direction


@pytest.mark.parametrize("prec", F16S, ids=PID.get)
@pytest.mark.parametrize("sign", [+1, -1])
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (6, 8, 10, 4), (8, 8, 8, 8)],
                         ids=lambda d: "x".join(map(str, d)))
def test_qtm(dims, sign, prec):
    kappa, mu = 0.1632, 0.45
    U = haar(dims, 811)
    psi = gauss(np.prod(dims) // 2, 812)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U, prec)
    out = lat.new_spinor(prec)
    tm.qtm_apply(lat, out, G, tm.spinor_import(lat, psi, prec), kappa, mu, THETA_AP, sign, prec)
    ref = oracle.qtm(dims, links_seen(U, prec), round_f16(psi), kappa, mu, THETA_AP, sign)
    assert site_rel_err(to_host(tm.spinor_export(lat, out, prec)), ref) <= QTM_TOL


def test_scalar_prod_reads_fp16():
    dims = (6, 8, 10, 4)
    lat = tm.Lattice(dims)
    a, b = gauss(lat.Vh, 821), gauss(lat.Vh, 822)
    ta, tb = tm.spinor_import(lat, a, tm.F16), tm.spinor_import(lat, b, tm.F16)
    ref = float(np.vdot(round_f16(a), round_f16(b)).real)
    assert abs(tm.scalar_prod_r(lat, ta, tb, tm.F16) - ref) <= 1e-12 * abs(ref) + 1e-9


def solve(dims, U, b, kappa, mu, inner):
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U)
    x = lat.new_spinor()
    tm.profile_enable(lat, True)
    it, res, ok = tm.cg_solve(lat, x, tm.spinor_import(lat, b), G, kappa, mu, THETA_AP, 1e-10, 5000, inner)
    n = {p: sum(tm.profile_read(lat, tmhop.profile_kind(p, m))[0] for m in range(4)) for p in range(6)}
    return to_host(tm.spinor_export(lat, x)), it, res, ok, n


def true_res(dims, U, x, b, kappa, mu):
    r = b - oracle.normal(dims, U, x, kappa, mu, THETA_AP)
    return np.linalg.norm(r) / np.linalg.norm(b)


CG_DIMS, CG_KAPPA = (8, 8, 8, 8), 0.1632
CG_MU = mu_of(CG_KAPPA, 0.0013)


@pytest.mark.parametrize("inner", F16S, ids=PID.get)
def test_cg_fp16_inner(inner):
    U = haar(CG_DIMS, 831)
    b = gauss(np.prod(CG_DIMS) // 2, 832)
    x, it, res, ok, n = solve(CG_DIMS, U, b, CG_KAPPA, CG_MU, inner)
    assert ok and res <= 1e-10
    assert n[inner] >= 4 * it and n[tm.F32] == n[tm.F32_R12] == 0
    other = tm.F16 if inner == tm.F16_R12 else tm.F16_R12
    assert n[other] == 0
    assert true_res(CG_DIMS, U, x, b, CG_KAPPA, CG_MU) <= 1.05e-10


def test_cg_fp16_two_row_falls_back_for_u3():
    V = int(np.prod(CG_DIMS))
    U = haar(CG_DIMS, 841) * np.exp(1j * fieldgen.rng(842).uniform(-0.5, 0.5, (4, V, 1, 1)))
    b = gauss(V // 2, 843)
    x, it, res, ok, n = solve(CG_DIMS, U, b, CG_KAPPA, CG_MU, tm.F16_R12)
    assert ok and res <= 1e-10
    assert n[tm.F16] >= 4 * it and n[tm.F16_R12] == 0
    assert true_res(CG_DIMS, U, x, b, CG_KAPPA, CG_MU) <= 1.05e-10


def test_cg_fp16_zero_source_and_restart():
    dims = (4, 6, 2, 6)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, haar(dims, 851))
    z = lat.new_spinor()
    x = lat.new_spinor()
    x.fill_(1.0)
    it, res, ok = tm.cg_solve(lat, x, z, G, CG_KAPPA, CG_MU, THETA_AP, 1e-10, 100, tm.F16)
    assert ok and it == 0 and float(x[:, :lat.Vh].abs().max()) == 0.0
    b = tm.spinor_import(lat, gauss(lat.Vh, 852))
    it, res, ok = tm.cg_solve(lat, x, b, G, CG_KAPPA, CG_MU, THETA_AP, 1e-10, 5000, tm.F16_R12)
    assert ok
    it2, res2, ok2 = tm.cg_solve(lat, x, b, G, CG_KAPPA, CG_MU, THETA_AP, 1e-10, 5000, tm.F16_R12)
    assert ok2 and it2 == 0


@pytest.mark.slow
def test_full_size_32x32x32x64_fp16_hop():
    """The 32^3x64 benchmark lattice, FP16 two-row storage: hop on the
    time-slice boundaries and random interior sites."""
    dims, kappa = QTM32["dims"], QTM32["kappa"]
    U = haar(dims, QTM32["seed"])
    Vh = np.prod(dims) // 2
    psi = gauss(Vh, 100 + QTM32["seed"])
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U, tm.F16_R12)
    x = tm.spinor_import(lat, psi, tm.F16_R12)
    out = lat.new_spinor(tm.F16_R12)
    g = fieldgen.rng(861)
    slab = dims[1] * dims[2] * dims[3] // 2
    sites = np.unique(np.concatenate([np.arange(slab), np.arange(Vh - slab, Vh),
                                      g.integers(0, Vh, 20000)]))
    Us = links_seen(U, tm.F16_R12)
    ps = round_f16(psi)
    for direction in ("eo", "oe"):
        tm.hop_apply(lat, direction, out, G, x, kappa, THETA_AP, tm.F16_R12)
        got = to_host(tm.spinor_export(lat, out, tm.F16_R12))[sites]
        ref = oracle.hop_sites(dims, direction, sites, Us, ps, kappa, THETA_AP)
        assert site_rel_err(got, ref) <= HOP_TOL
