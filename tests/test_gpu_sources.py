"""Sources the random Gaussian workloads do not cover, through every solver
code: a point source (one spin-colour component at one site), and sources
scaled far from unit size.  What is unique is checked: the true residual
under the oracle's operator, and for the scaled sources that the solution
scales with the source (the system is linear)."""

import numpy as np
import pytest

import oracle
import paper_1311_4521_amd as tm
from helpers import THETA_AP, gauss, haar, mu_of

pytestmark = pytest.mark.gpu

CODES = [tm.F64, tm.F32, tm.F64_R12, tm.F32_R12, tm.F16, tm.F16_R12]
IDS = {tm.F64: "f64", tm.F32: "f32", tm.F64_R12: "f64r12", tm.F32_R12: "f32r12",
       tm.F16: "f16", tm.F16_R12: "f16r12"}
DIMS, KAPPA = (8, 8, 8, 8), 0.1632
MU = mu_of(KAPPA, 0.0013)


def solve(U, b, inner):
    lat = tm.Lattice(DIMS)
    G = tm.gauge_import(lat, U)
    x = lat.new_spinor()
    it, res, ok = tm.cg_solve(lat, x, tm.spinor_import(lat, b), G, KAPPA, MU, THETA_AP, 1e-10, 5000, inner)
    return tm.spinor_export(lat, x).cpu().numpy(), it, res, ok


def oracle_res(U, x, b):
    r = b - oracle.normal(DIMS, U, x, KAPPA, MU, THETA_AP)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.parametrize("inner", CODES, ids=IDS.get)
def test_point_source(inner):
    U = haar(DIMS, 901)
    b = np.zeros((np.prod(DIMS) // 2, 4, 3), dtype=np.complex128)
    b[1037, 2, 1] = 1.0
    x, it, res, ok = solve(U, b, inner)
    assert ok and res <= 1e-10
    assert oracle_res(U, x, b) <= 1.05e-10


@pytest.mark.parametrize("inner", CODES, ids=IDS.get)
@pytest.mark.parametrize("s", [1e-40, 1e30], ids=["1e-40", "1e30"])
def test_source_magnitude(inner, s):
    """1e-40 lies below FP32's and FP16's ranges, 1e30 above FP16's: the
    inner solves see the residual scaled to unit size either way."""
    U = haar(DIMS, 902)
    b = gauss(np.prod(DIMS) // 2, 903)
    x1, _, res1, ok1 = solve(U, b, inner)
    xs, _, ress, oks = solve(U, s * b, inner)
    assert ok1 and oks and ress <= 1e-10
    assert oracle_res(U, xs, s * b) <= 1.05e-10
    # both solutions solve their systems to 1e-10, so they agree to about
    # cond * 1e-10; the condition number of this system is below 1e3
    assert np.linalg.norm(xs / s - x1) <= 1e-6 * np.linalg.norm(x1)


@pytest.mark.parametrize("inner", CODES, ids=IDS.get)
def test_iteration_cap(inner):
    """With too few iterations allowed every code reports non-convergence,
    stays within the cap and returns a finite true residual."""
    U = haar(DIMS, 904)
    b = gauss(np.prod(DIMS) // 2, 905)
    x, it, res, ok = solve_capped(U, b, inner, 3)
    assert not ok and 1 <= it <= 3
    assert np.isfinite(res) and 1e-10 < res < 1.0
    assert np.all(np.isfinite(x))
    assert abs(oracle_res(U, x, b) - res) <= 1e-6 * res


def solve_capped(U, b, inner, max_iter):
    lat = tm.Lattice(DIMS)
    G = tm.gauge_import(lat, U)
    x = lat.new_spinor()
    it, res, ok = tm.cg_solve(lat, x, tm.spinor_import(lat, b), G, KAPPA, MU, THETA_AP, 1e-10, max_iter, inner)
    return tm.spinor_export(lat, x).cpu().numpy(), it, res, ok
