"""The t-marching hop kernel (TMH_TRAVERSAL_TMARCH) against the oracle and
against the one-site-per-lane kernel.

Both kernels add the same 8 terms in the same order, so the FP64 and FP32
hop outputs must agree to a few units in the last place whatever the step
count (1e-14 FP64, 1e-6 FP32 per site: the compiler may fuse multiply-adds
differently in the two kernels; in FP16 storage it fuses the conversions
too, so only the oracle bar applies); the oracle bar is that of every hop
(1e-13 FP64, 1e-5 FP32, the FP16 bar on FP16-rounded inputs).  The CG recursions take the fused
epilogues of the t-march (modes 1-4) and must reach the oracle-certified
true residual.  Lattices: every slice of 256 pairs or a multiple, T = 2
(both time neighbours are the same site), twisted phases in all
directions, and every step count that divides T."""

import numpy as np
import pytest
import torch

import fieldgen
import oracle
import paper_1311_4521_amd as tm
from helpers import QTM32, THETA_AP, gauss, haar, mu_of, site_rel_err

pytestmark = pytest.mark.gpu

THETA = (0.5, 0.25, -0.3, 0.7)
TOL = {tm.F64: 1e-13, tm.F64_R12: 1e-13, tm.F32: 1e-5, tm.F32_R12: 1e-5}
SAME = {tm.F64: 1e-14, tm.F64_R12: 1e-14, tm.F32: 1e-6, tm.F32_R12: 1e-6}
SHAPES = [(8, 8, 8, 8), (2, 8, 8, 8), (6, 8, 8, 16), (4, 16, 8, 4), (10, 4, 8, 16), (4, 2, 16, 16)]


def f16_round(a):
    f = lambda v: v.astype(np.float16).astype(np.float64)
    return f(a.real) + 1j * f(a.imag)


def divisors(n):
    return [d for d in range(1, n + 1) if n % d == 0]


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("dims", SHAPES, ids=lambda d: "x".join(map(str, d)))
def test_tmarch_hop_every_code_and_step_count(dims):
    kappa = 0.13
    V = int(np.prod(dims))
    U = fieldgen.gauge_haar(dims, 80 + V % 97)
    lat = tm.Lattice(dims)
    Uh = f16_round(U)
    Uh12 = Uh.copy()
    Uh12[..., 2, :] = np.conj(np.cross(Uh[..., 0, :], Uh[..., 1, :]))
    for direction, seed in (("eo", 3), ("oe", 4)):
        psi = fieldgen.spinor_gauss(V // 2, seed + V % 89)
        ref = oracle.hop(dims, direction, U, psi, kappa, THETA)
        ref16 = {tm.F16: oracle.hop(dims, direction, Uh, f16_round(psi), kappa, THETA),
                 tm.F16_R12: oracle.hop(dims, direction, Uh12, f16_round(psi), kappa, THETA)}
        for prec in (tm.F64, tm.F64_R12, tm.F32, tm.F32_R12, tm.F16, tm.F16_R12):
            G = tm.gauge_import(lat, U, prec)
            x = tm.spinor_import(lat, psi, prec)
            lat.traversal = 0
            base = lat.new_spinor(prec)
            tm.hop_apply(lat, direction, base, G, x, kappa, THETA, prec)
            for steps in divisors(dims[0]):
                lat.traversal = tm.TMARCH(steps)
                out = lat.new_spinor(prec)
                tm.hop_apply(lat, direction, out, G, x, kappa, THETA, prec)
                name = (direction, tm.tmhop.PREC_NAMES[prec], steps)
                got = host(tm.spinor_export(lat, out, prec))
                if prec in TOL:
                    assert site_rel_err(got, host(tm.spinor_export(lat, base, prec))) <= SAME[prec], name
                    assert site_rel_err(got, ref) <= TOL[prec], name
                else:
                    assert site_rel_err(got, ref16[prec]) <= 2.0 ** -11 + 2e-6, name


def test_tmarch_rejected_where_it_does_not_tile():
    lat = tm.Lattice((8, 4, 4, 4))          # 32 pairs per slice
    with pytest.raises(tm.TmhError):
        lat.traversal = tm.TMARCH(2)
    lat2 = tm.Lattice((6, 8, 8, 8))
    with pytest.raises(tm.TmhError):
        lat2.traversal = tm.TMARCH(4)       # does not divide T
    lat2.traversal = tm.TMARCH(3)
    assert lat2.traversal == tm.TMARCH(3)


@pytest.mark.parametrize("inner", [tm.F64, tm.F32, tm.F16_R12], ids=["f64", "f32", "f16r12"])
@pytest.mark.parametrize("steps", [1, 4, 8])
def test_tmarch_qtm_and_cg(steps, inner):
    """Qhat (modes 0 and 1) equal to the one-site-per-lane kernel's to 1e-14;
    the CG recursions (modes 0, 2, 3/4) reach the oracle-certified residual
    in about the same number of iterations."""
    dims, kappa = (8, 8, 8, 16), 0.1632
    mu = mu_of(kappa, 0.0013)
    U = haar(dims, 811)
    b = gauss(int(np.prod(dims)) // 2, 812)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U)
    tb = tm.spinor_import(lat, b)
    lat.traversal = 0
    q0 = lat.new_spinor()
    tm.qtm_apply(lat, q0, G, tb, kappa, mu, THETA_AP, +1)
    x0 = lat.new_spinor()
    it0, _, ok0 = tm.cg_solve(lat, x0, tb, G, kappa, mu, THETA_AP, 1e-10, 2000, inner)
    lat.traversal = tm.TMARCH(steps)
    q = lat.new_spinor()
    tm.qtm_apply(lat, q, G, tb, kappa, mu, THETA_AP, +1)
    assert site_rel_err(host(tm.spinor_export(lat, q)), host(tm.spinor_export(lat, q0))) <= 1e-14
    x = lat.new_spinor()
    it, res, ok = tm.cg_solve(lat, x, tb, G, kappa, mu, THETA_AP, 1e-10, 2000, inner)
    assert ok0 and ok and res <= 1e-10 and abs(it - it0) <= 2
    r = b - oracle.normal(dims, U, host(tm.spinor_export(lat, x)), kappa, mu, THETA_AP)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.05e-10


def test_tmarch_cg_repeats_bitwise():
    """The fused norms of the t-march sum in a fixed order: two solves give
    bitwise the same solution."""
    dims, kappa = (8, 8, 8, 16), 0.1632
    mu = mu_of(kappa, 0.0013)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, haar(dims, 821))
    tb = tm.spinor_import(lat, gauss(lat.Vh, 822))
    lat.traversal = tm.TMARCH(4)
    outs = []
    for _ in range(2):
        x = lat.new_spinor()
        it, res, ok = tm.cg_solve(lat, x, tb, G, kappa, mu, THETA_AP, 1e-10, 2000)
        assert ok
        outs.append((it, res, x))
    assert outs[0][0] == outs[1][0] and outs[0][1] == outs[1][1] and torch.equal(outs[0][2], outs[1][2])


@pytest.mark.slow
def test_tmarch_full_size_32x32x32x64():
    """The benchmark lattice: every t-march step count the autotuner tries
    there gives the one-site-per-lane kernel's output to 1e-14 per site,
    which matches the oracle on every boundary time-slice and 20,000 random
    sites."""
    dims, kappa = QTM32["dims"], QTM32["kappa"]
    U = haar(dims, QTM32["seed"])
    Vh = int(np.prod(dims)) // 2
    psi = gauss(Vh, 100 + QTM32["seed"])
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U)
    x = tm.spinor_import(lat, psi)
    g = fieldgen.rng(37)
    slab = dims[1] * dims[2] * dims[3] // 2
    sites = np.unique(np.concatenate([np.arange(slab), np.arange(Vh - slab, Vh), g.integers(0, Vh, 20000)]))
    for direction in ("eo", "oe"):
        lat.traversal = 16
        base = lat.new_spinor()
        tm.hop_apply(lat, direction, base, G, x, kappa, THETA_AP)
        ref = oracle.hop_sites(dims, direction, sites, U, psi, kappa, THETA_AP)
        assert site_rel_err(host(tm.spinor_export(lat, base))[sites], ref) <= 1e-13
        for steps in (4, 8, 16, 32):
            lat.traversal = tm.TMARCH(steps)
            out = lat.new_spinor()
            tm.hop_apply(lat, direction, out, G, x, kappa, THETA_AP)
            got = host(tm.spinor_export(lat, out))
            assert site_rel_err(got[sites], ref) <= 1e-13, (direction, steps)
            assert site_rel_err(got, host(tm.spinor_export(lat, base))) <= 1e-14, (direction, steps)
