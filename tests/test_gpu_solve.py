"""Full-lattice solve M x = b through the even-odd split (tmh_solve_full),
certified with the oracle's full-lattice operator (which never splits the
lattice) and, on 2^4, with numpy.linalg.solve on the dense matrix."""

import numpy as np
import pytest

import dense
import fieldgen
import oracle
import paper_1311_4521_amd as tm
from helpers import THETA_AP, haar, mu_of

pytestmark = pytest.mark.gpu


def solve(dims, U, b, kappa, mu, inner=tm.F64, tol=1e-11):
    ev, od = dense.parity_sites(dims, 0), dense.parity_sites(dims, 1)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U)
    be, bo = tm.spinor_import(lat, b[ev]), tm.spinor_import(lat, b[od])
    xe, xo = lat.new_spinor(), lat.new_spinor()
    it, res, ok = tm.solve_full(lat, xe, xo, be, bo, G, kappa, mu, THETA_AP, tol, 5000, inner)
    x = np.empty_like(b)
    x[ev] = tm.spinor_export(lat, xe).cpu().numpy()
    x[od] = tm.spinor_export(lat, xo).cpu().numpy()
    return x, it, res, ok


def test_solve_full_dense_2x2x2x2():
    dims, kappa, mu = (2, 2, 2, 2), 0.1632, mu_of(0.1632, 0.0013)
    U = haar(dims, 401)
    b = fieldgen.spinor_gauss(16, 402)
    x, it, res, ok = solve(dims, U, b, kappa, mu)
    assert ok
    M = dense.full_operator(dims, U, kappa, mu, THETA_AP)
    xr = np.linalg.solve(M, b.ravel())
    assert np.linalg.norm(x.ravel() - xr) / np.linalg.norm(xr) < 1e-9


@pytest.mark.parametrize("inner", [tm.F64, tm.F32, tm.F64_R12, tm.F32_R12],
                         ids=["f64", "f32", "f64r12", "f32r12"])
@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 8, 10, 4)], ids=lambda d: "x".join(map(str, d)))
def test_solve_full_residual(dims, inner):
    kappa, mu = 0.1632, mu_of(0.1632, 0.0013)
    U = haar(dims, 411)
    b = fieldgen.spinor_gauss(int(np.prod(dims)), 412)
    x, it, res, ok = solve(dims, U, b, kappa, mu, inner)
    assert ok and res <= 1e-11
    r = b - oracle.full_operator(dims, U, x, kappa, mu, THETA_AP)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 1e-9
