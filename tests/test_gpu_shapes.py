"""A seeded sweep of lattice shapes against the oracle: every extent even
from 2 to 12 (and a few long ones), both hop directions, every storage code,
with twisted boundary phases in all four directions.  Shapes whose (t, x)
planes hold a multiple of 64 sites and whose T is a multiple of 8 take the
x-group traversal by default (the first three, whose half volume is also a
multiple of 2048 sites); the others take even-odd order."""

import numpy as np
import pytest

import fieldgen
import oracle
import paper_1311_4521_amd as tm
from helpers import site_rel_err

pytestmark = pytest.mark.gpu

THETA = (0.5, 0.25, -0.3, 0.7)
TOL = {tm.F64: 1e-13, tm.F64_R12: 1e-13, tm.F32: 1e-5, tm.F32_R12: 1e-5}


def shapes():
    g = fieldgen.rng(4242)
    out = [(8, 4, 4, 32), (16, 4, 2, 64), (8, 8, 8, 16), (2, 12, 2, 2), (12, 2, 12, 2)]
    while len(out) < 16:
        d = tuple(int(v) for v in 2 * g.integers(1, 7, 4))
        if d not in out:
            out.append(d)
    return out


def f16_round(a):
    f = lambda v: v.astype(np.float16).astype(np.float64)
    return f(a.real) + 1j * f(a.imag)


@pytest.mark.parametrize("dims", shapes(), ids=lambda d: "x".join(map(str, d)))
def test_hop_every_code(dims):
    kappa = 0.13
    V = int(np.prod(dims))
    U = fieldgen.gauge_haar(dims, 60 + V % 97)
    lat = tm.Lattice(dims)
    for direction, seed in (("eo", 1), ("oe", 2)):
        psi = fieldgen.spinor_gauss(V // 2, seed + V % 89)
        ref = oracle.hop(dims, direction, U, psi, kappa, THETA)
        for prec in (tm.F64, tm.F64_R12, tm.F32, tm.F32_R12):
            G = tm.gauge_import(lat, U, prec)
            out = lat.new_spinor(prec)
            tm.hop_apply(lat, direction, out, G, tm.spinor_import(lat, psi, prec), kappa, THETA, prec)
            got = tm.spinor_export(lat, out, prec).cpu().numpy()
            assert site_rel_err(got, ref) <= TOL[prec], (direction, tm.tmhop.PREC_NAMES[prec])
        # FP16: the oracle takes the rounded inputs the kernel reads
        Uh = f16_round(U)
        Uh12 = Uh.copy()
        Uh12[..., 2, :] = np.conj(np.cross(Uh[..., 0, :], Uh[..., 1, :]))
        for prec, Us in ((tm.F16, Uh), (tm.F16_R12, Uh12)):
            ref16 = oracle.hop(dims, direction, Us, f16_round(psi), kappa, THETA)
            G = tm.gauge_import(lat, U, prec)
            out = lat.new_spinor(prec)
            tm.hop_apply(lat, direction, out, G, tm.spinor_import(lat, psi, prec), kappa, THETA, prec)
            got = tm.spinor_export(lat, out, prec).cpu().numpy()
            assert site_rel_err(got, ref16) <= 2.0 ** -11 + 2e-6, (direction, tm.tmhop.PREC_NAMES[prec])


@pytest.mark.parametrize("dims", shapes()[:8], ids=lambda d: "x".join(map(str, d)))
def test_qtm_f64(dims):
    kappa, mu = 0.15, 0.3
    V = int(np.prod(dims))
    U = fieldgen.gauge_haar(dims, 70 + V % 97)
    psi = fieldgen.spinor_gauss(V // 2, 71)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U)
    for sign in (+1, -1):
        out = lat.new_spinor()
        tm.qtm_apply(lat, out, G, tm.spinor_import(lat, psi), kappa, mu, THETA, sign)
        ref = oracle.qtm(dims, U, psi, kappa, mu, THETA, sign)
        assert site_rel_err(tm.spinor_export(lat, out).cpu().numpy(), ref) <= 1e-13
