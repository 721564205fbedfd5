"""Bitwise reproducibility on the GPU: every kernel has one writer per output
and every reduction sums in a fixed order, so repeating a call on the same
inputs must give identical bits (a race would show up here as a difference).
Covers the gauge-link force and every solver variant; the plain hop, Qtm and
FP64 CG are covered in test_gpu_parity.py."""

import numpy as np
import pytest
import torch

import paper_1311_4521_amd as tm
from helpers import THETA_AP, gauss, haar, mu_of

pytestmark = pytest.mark.gpu

DIMS = (8, 8, 8, 8)
KAPPA = 0.1632
MU = mu_of(KAPPA, 0.0013)


def setup():
    lat = tm.Lattice(DIMS)
    G = tm.gauge_import(lat, haar(DIMS, 901))
    a = tm.spinor_import(lat, gauss(lat.Vh, 902))
    b = tm.spinor_import(lat, gauss(lat.Vh, 903))
    return lat, G, a, b


@pytest.mark.parametrize("kind", ["su3", "euclid"])
def test_force_repeats_bitwise(kind):
    lat, G, a, b = setup()
    outs = []
    for _ in range(2):
        F = lat.new_gauge(zero=True)
        tm.hop_force(lat, "eo", F, G, a, b, KAPPA, THETA_AP, 0.5, kind)
        tm.qtm_force(lat, F, G, a, b, KAPPA, MU, THETA_AP, -1, 1.0, kind)
        outs.append(F)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("inner", [tm.F64_R12, tm.F32, tm.F32_R12, tm.F16, tm.F16_R12],
                         ids=["f64r12", "f32", "f32r12", "f16", "f16r12"])
def test_solver_repeats_bitwise(inner):
    lat, G, a, _ = setup()
    res = []
    for _ in range(2):
        x = lat.new_spinor()
        res.append((tm.cg_solve(lat, x, a, G, KAPPA, MU, THETA_AP, 1e-10, 5000, inner), x))
    assert res[0][0] == res[1][0]
    assert res[0][0][2]
    assert torch.equal(res[0][1], res[1][1])


def test_multi_rhs_hop_repeats_bitwise():
    lat, G, _, _ = setup()
    X = lat.new_spinors(5)
    for r in range(5):
        tm.spinor_import(lat, gauss(lat.Vh, 910 + r), out=X[r])
    outs = []
    for shape in ("128x4", "128x4"):
        Y = lat.new_spinors(5)
        tm.hop_apply_mrhs(lat, "oe", Y, G, X, KAPPA, THETA_AP, tm.F64, shape)
        outs.append(Y)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
