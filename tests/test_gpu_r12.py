"""Two-row link storage (TMH_F64_R12, TMH_F32_R12) on the GPU against the
oracle, which always applies the full 9-entry links.

For special unitary links the third row equals the complex conjugate of the
cross product of the first two, so the compressed operators are the same
operators: bars 1e-13 (FP64) and 1e-5 (FP32) per-site relative error, as for
the full storage.  The solver with a two-row inner code runs its recursion
on a two-row copy when the links pass its check and keeps 9 entries
otherwise; both branches are exercised here, the branch taken read from the
launch-kind counters."""

import numpy as np
import pytest
import torch

import fieldgen
import oracle
import paper_1311_4521_amd as tm
from paper_1311_4521_amd import tmhop
from helpers import HOP8, QTM32, THETA_AP, gauss, haar, mu_of, site_rel_err

pytestmark = pytest.mark.gpu

R12 = [tm.F64_R12, tm.F32_R12]
TOL = {tm.F64_R12: 1e-13, tm.F32_R12: 1e-5}
PID = {tm.F64_R12: "f64r12", tm.F32_R12: "f32r12"}
SMALL = [(2, 2, 2, 2), (6, 2, 4, 2), (4, 6, 2, 6), (6, 8, 10, 4), (8, 6, 4, 10)]
THETAS = [THETA_AP, (0.5, 0.25, -0.3, 0.7)]


def to_host(t):
    return t.detach().cpu().numpy()


def run_hop(dims, U, psi, direction, kappa, theta, prec):
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U, prec)
    x = tm.spinor_import(lat, psi, prec)
    out = lat.new_spinor(prec)
    tm.hop_apply(lat, direction, out, G, x, kappa, theta, prec)
    return to_host(tm.spinor_export(lat, out, prec))


def test_storage_size_and_roundtrip():
    dims = (4, 6, 2, 6)
    U = haar(dims, 701)
    lat = tm.Lattice(dims)
    assert lat.gauge_bytes(tm.F64_R12) * 3 == lat.gauge_bytes(tm.F64) * 2
    assert lat.gauge_bytes(tm.F32_R12) * 3 == lat.gauge_bytes(tm.F32) * 2
    assert lat.spinor_bytes(tm.F64_R12) == lat.spinor_bytes(tm.F64)
    G = tm.gauge_import(lat, U, tm.F64_R12)
    assert tuple(G.shape) == (2, 4, 6, lat.S, 2)
    back = to_host(tm.gauge_export(lat, G, tm.F64_R12))
    # stored rows come back exactly, the rebuilt row to rounding
    assert np.array_equal(back[:, :, :2], U[:, :, :2])
    assert np.abs(back - U).max() <= 1e-14
    back32 = to_host(tm.gauge_export(lat, tm.gauge_import(lat, U, tm.F32_R12), tm.F32_R12))
    assert np.abs(back32 - U).max() <= 1e-6


@pytest.mark.parametrize("prec", R12, ids=PID.get)
@pytest.mark.parametrize("direction", ["eo", "oe"])
def test_hop_8x8x8x8(direction, prec):
    dims, kappa = HOP8["dims"], HOP8["kappa"]
    U = haar(dims, HOP8["seed"])
    psi = gauss(np.prod(dims) // 2, 100 + HOP8["seed"])
    ref = oracle.hop(dims, direction, U, psi, kappa, THETA_AP)
    assert site_rel_err(run_hop(dims, U, psi, direction, kappa, THETA_AP, prec), ref) <= TOL[prec]


@pytest.mark.parametrize("prec", R12, ids=PID.get)
@pytest.mark.parametrize("theta", THETAS, ids=["ap", "twisted"])
@pytest.mark.parametrize("dims", SMALL, ids=lambda d: "x".join(map(str, d)))
def test_hop_small_lattices(dims, theta, prec):
    kappa = 0.137
    U = haar(dims, 7)
    for direction, seed in (("eo", 8), ("oe", 9)):
        psi = gauss(np.prod(dims) // 2, seed)
        ref = oracle.hop(dims, direction, U, psi, kappa, theta)
        assert site_rel_err(run_hop(dims, U, psi, direction, kappa, theta, prec), ref) <= TOL[prec]


@pytest.mark.parametrize("prec", R12, ids=PID.get)
@pytest.mark.parametrize("sign", [+1, -1])
@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (6, 8, 10, 4), (8, 8, 8, 8)],
                         ids=lambda d: "x".join(map(str, d)))
def test_qtm(dims, sign, prec):
    kappa, mu = 0.1632, 0.45
    U = haar(dims, 711)
    psi = gauss(np.prod(dims) // 2, 712)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U, prec)
    out = lat.new_spinor(prec)
    tm.qtm_apply(lat, out, G, tm.spinor_import(lat, psi, prec), kappa, mu, THETA_AP, sign, prec)
    ref = oracle.qtm(dims, U, psi, kappa, mu, THETA_AP, sign)
    assert site_rel_err(to_host(tm.spinor_export(lat, out, prec)), ref) <= TOL[prec]


def test_traversals_agree_with_two_row_links():
    dims, kappa = (8, 8, 8, 16), 0.1632
    U = haar(dims, 721)
    psi = gauss(int(np.prod(dims)) // 2, 722)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U, tm.F64_R12)
    x = tm.spinor_import(lat, psi, tm.F64_R12)
    ref = oracle.hop(dims, "oe", U, psi, kappa, THETA_AP)
    first = None
    for xg in (0, 1, 2, 4, 8, tm.XSLAB):
        lat.traversal = xg
        out = lat.new_spinor(tm.F64_R12)
        tm.hop_apply(lat, "oe", out, G, x, kappa, THETA_AP, tm.F64_R12)
        if first is None:
            first = out
            assert site_rel_err(to_host(tm.spinor_export(lat, out)), ref) <= 1e-13
        else:
            assert torch.equal(out, first), xg


def solve(dims, U, b, kappa, mu, inner):
    """CG with launch timing on; returns the solution, the result and the
    hop launches per precision code."""
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U)
    x = lat.new_spinor()
    tm.profile_enable(lat, True)
    it, res, ok = tm.cg_solve(lat, x, tm.spinor_import(lat, b), G, kappa, mu, THETA_AP, 1e-10, 5000, inner)
    n = {p: sum(tm.profile_read(lat, tmhop.profile_kind(p, m))[0] for m in range(4))
         for p in (tm.F64, tm.F32, tm.F64_R12, tm.F32_R12)}
    return to_host(tm.spinor_export(lat, x)), it, res, ok, n


def true_res(dims, U, x, b, kappa, mu):
    r = b - oracle.normal(dims, U, x, kappa, mu, THETA_AP)
    return np.linalg.norm(r) / np.linalg.norm(b)


def u3_links(dims, seed):
    """Haar SU(3) links times a random phase each: unitary, det != 1."""
    V = int(np.prod(dims))
    return haar(dims, seed) * np.exp(1j * fieldgen.rng(seed + 1).uniform(-0.5, 0.5, (4, V, 1, 1)))


CG_DIMS, CG_KAPPA = (8, 8, 8, 8), 0.1632
CG_MU = mu_of(CG_KAPPA, 0.0013)


@pytest.mark.parametrize("inner", [tm.F64_R12, tm.F32_R12], ids=PID.get)
def test_cg_on_two_row_links(inner):
    """SU(3) links: every launch of the solve, the FP64 true residuals
    included, reads a two-row copy, and the solution solves the oracle's
    system (which applies the full 9-entry links); the FP64 variant matches
    the 9-entry FP64 solve."""
    U = haar(CG_DIMS, 731)
    b = gauss(np.prod(CG_DIMS) // 2, 732)
    x, it, res, ok, n = solve(CG_DIMS, U, b, CG_KAPPA, CG_MU, inner)
    assert ok and res <= 1e-10
    assert n[inner] >= 4 * it
    assert n[tm.F64] == 0 and n[tm.F32] == 0
    assert true_res(CG_DIMS, U, x, b, CG_KAPPA, CG_MU) <= 1.05e-10
    if inner == tm.F64_R12:
        xf, itf, _, okf, nf = solve(CG_DIMS, U, b, CG_KAPPA, CG_MU, tm.F64)
        assert okf and nf[tm.F64_R12] == 0 and abs(it - itf) <= 1
        assert np.linalg.norm(x - xf) / np.linalg.norm(xf) <= 1e-9


@pytest.mark.parametrize("inner", [tm.F64_R12, tm.F32_R12], ids=PID.get)
def test_cg_keeps_full_links_for_u3(inner):
    """Unitary links outside SU(3): the rebuilt row would be wrong, so the
    solver keeps all 9 entries and still solves the oracle's system."""
    U = u3_links(CG_DIMS, 741)
    b = gauss(np.prod(CG_DIMS) // 2, 743)
    x, it, res, ok, n = solve(CG_DIMS, U, b, CG_KAPPA, CG_MU, inner)
    assert ok and res <= 1e-10
    full = tm.F64 if inner == tm.F64_R12 else tm.F32
    assert n[full] >= 4 * it and n[inner] == 0
    assert true_res(CG_DIMS, U, x, b, CG_KAPPA, CG_MU) <= 1.05e-10


def test_plain_f32_inner_keeps_nine_entries():
    U = haar(CG_DIMS, 731)
    b = gauss(np.prod(CG_DIMS) // 2, 732)
    x, it, res, ok, n = solve(CG_DIMS, U, b, CG_KAPPA, CG_MU, tm.F32)
    assert ok and n[tm.F32] > 0 and n[tm.F32_R12] == 0


def test_multi_rhs_rejects_two_row_codes():
    dims = (4, 4, 4, 4)
    lat = tm.Lattice(dims)
    G12 = tm.gauge_import(lat, haar(dims, 751), tm.F64_R12)
    ins, outs = lat.new_spinors(2), lat.new_spinors(2)
    with pytest.raises(tm.TmhError) as e:
        tm.hop_apply_mrhs(lat, "eo", outs, G12, ins, 0.16, THETA_AP, tm.F64_R12)
    assert e.value.status == tmhop.TMH_ERR_UNSUPPORTED


def test_autotune_hop_two_row_cache(tmp_path):
    dims = (8, 8, 8, 16)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, haar(dims, 761), tm.F32_R12)
    cache = str(tmp_path / "hop.txt")
    xg, us = tm.autotune_hop(lat, G, tm.F32_R12, cache)
    assert us > 0 and lat.traversal == xg
    assert open(cache).read().split()[1:4] == ["8x8x8x16", "f32r12", "hop"]


@pytest.mark.slow
def test_full_size_32x32x32x64_two_row_hop():
    """The 32^3x64 benchmark lattice with FP64 two-row links: hop on sampled
    sites (the time-slice boundaries and random interior sites)."""
    dims, kappa = QTM32["dims"], QTM32["kappa"]
    U = haar(dims, QTM32["seed"])
    Vh = np.prod(dims) // 2
    psi = gauss(Vh, 100 + QTM32["seed"])
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U, tm.F64_R12)
    x = tm.spinor_import(lat, psi)
    out = lat.new_spinor()
    g = fieldgen.rng(771)
    slab = dims[1] * dims[2] * dims[3] // 2
    sites = np.unique(np.concatenate([np.arange(slab), np.arange(Vh - slab, Vh),
                                      g.integers(0, Vh, 20000)]))
    for direction in ("eo", "oe"):
        tm.hop_apply(lat, direction, out, G, x, kappa, THETA_AP, tm.F64_R12)
        got = to_host(tm.spinor_export(lat, out))[sites]
        ref = oracle.hop_sites(dims, direction, sites, U, psi, kappa, THETA_AP)
        assert site_rel_err(got, ref) <= 1e-13
