"""Batched path: the multi-right-hand-side hop of every tile shape against
the oracle, the batched CG over several lattices (with and without graph
replay) certified per system with the oracle's operator, and the autotuner."""

import os

import numpy as np
import pytest
import torch

import oracle
import paper_1311_4521_amd as tm
from helpers import THETA_AP, gauss, haar, mu_of, round_f32, site_rel_err

pytestmark = pytest.mark.gpu

TWIST = (0.5, 0.25, -0.3, 0.7)


def host(t):
    return t.detach().cpu().numpy()


def import_many(lat, fields, prec=tm.F64):
    out = lat.new_spinors(len(fields), prec)
    for r, f in enumerate(fields):
        tm.spinor_import(lat, f, prec, out=out[r])
    return out


@pytest.mark.parametrize("prec", [tm.F64, tm.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape", list(tm.tmhop.SHAPES))
@pytest.mark.parametrize("dims,nrhs", [((6, 8, 10, 4), 3), ((8, 8, 8, 8), 12), ((2, 2, 2, 2), 5),
                                       ((8, 6, 16, 16), 12), ((16, 4, 16, 32), 5), ((6, 4, 8, 4), 7)],
                         ids=["6x8x10x4-3", "8x8x8x8-12", "2x2x2x2-5", "8x6x16x16-12", "16x4x16x32-5",
                              "6x4x8x4-7"])
def test_hop_mrhs_matches_oracle(dims, nrhs, shape, prec):
    """The last two lattices take the x-group tile order (whole (t, x)
    planes of 128 and 256 sites, T a multiple of 8) for the shapes whose
    tiles divide the plane; the others take even-odd order."""
    kappa = 0.15
    U = haar(dims, 501)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U, prec)
    psis = [gauss(lat.Vh, 510 + r) for r in range(nrhs)]
    inp = import_many(lat, psis, prec)
    out = lat.new_spinors(nrhs, prec)
    tol = 1e-13 if prec == tm.F64 else 1e-5
    sid = tm.tmhop.SHAPES[shape]
    if sid in tm.tmhop.TMARCH_SHAPES and (dims[1] * dims[2] * dims[3] // 2) % (64 if sid in (15, 16) else 256):
        with pytest.raises(tm.TmhError) as e:
            tm.hop_apply_mrhs(lat, "eo", out, G, inp, kappa, TWIST, prec, shape)
        assert e.value.status == tm.tmhop.TMH_ERR_UNSUPPORTED
        return
    for direction in ("eo", "oe"):
        tm.hop_apply_mrhs(lat, direction, out, G, inp, kappa, TWIST, prec, shape)
        for r in range(nrhs):
            ref = oracle.hop(dims, direction, U, psis[r], kappa, TWIST)
            got = host(tm.spinor_export(lat, out[r], prec))
            assert site_rel_err(got, ref) <= tol, (direction, r)


def batch_problem():
    kappa, mu = 0.1632, mu_of(0.1632, 0.0013)
    specs = [((8, 8, 8, 8), 3, 521), ((6, 8, 10, 4), 5, 531), ((4, 4, 4, 4), 2, 541), ((8, 4, 16, 16), 2, 551)]
    members, host_data = [], []
    for dims, nrhs, seed in specs:
        lat = tm.Lattice(dims)
        U = haar(dims, seed)
        bs = [gauss(lat.Vh, seed + 1 + r) for r in range(nrhs)]
        members.append(dict(lat=lat, x=lat.new_spinors(nrhs), b=import_many(lat, bs),
                            gauge=tm.gauge_import(lat, U), kappa=kappa, mu=mu, theta=THETA_AP))
        host_data.append((dims, U, bs))
    return members, host_data, kappa, mu


@pytest.mark.parametrize("use_graph", [False, True], ids=["eager", "graph"])
def test_batch_cg_certified(use_graph):
    members, host_data, kappa, mu = batch_problem()
    it, res, ok = tm.batch_cg_solve(members, 1e-10, 2000, -1, use_graph)
    assert ok and len(it) == 12 and max(res) <= 1e-10
    k = 0
    for m, (dims, U, bs) in zip(members, host_data):
        for r, b in enumerate(bs):
            x = host(tm.spinor_export(m["lat"], m["x"][r]))
            rr = b - oracle.normal(dims, U, x, kappa, mu, THETA_AP)
            assert np.linalg.norm(rr) / np.linalg.norm(b) <= 1.05e-10, (dims, r)
            # the same system solved alone
            lat = m["lat"]
            x1 = lat.new_spinor()
            it1, res1, ok1 = tm.cg_solve(lat, x1, m["b"][r].contiguous(), m["gauge"], kappa, mu,
                                         THETA_AP, 1e-10, 2000)
            assert ok1 and abs(it1 - it[k]) <= 2
            assert float((x1 - m["x"][r]).norm() / x1.norm()) < 1e-7
            k += 1


def test_batch_graph_replays_match_eager():
    """Graph replay (several replays per solve, host work between them) gives
    bitwise the same solutions and counts as eager launches."""
    outs = []
    for use_graph in (False, True, True):
        members, _, _, _ = batch_problem()
        it, res, ok = tm.batch_cg_solve(members, 1e-10, 2000, 2, use_graph)
        assert ok
        outs.append((it, res, [m["x"].clone() for m in members]))
    for o in outs[1:]:
        assert o[0] == outs[0][0] and o[1] == outs[0][1]
        for a, b in zip(o[2], outs[0][2]):
            assert torch.equal(a, b)


@pytest.mark.parametrize("use_graph", [False, True], ids=["eager", "graph"])
def test_batch_nonzero_start(use_graph):
    """A start vector that is not zero in one system takes the true-residual
    path for the whole batch: restarting from the solutions takes no
    iterations, and a perturbed start converges again to the oracle's
    solution."""
    members, host_data, kappa, mu = batch_problem()
    it, res, ok = tm.batch_cg_solve(members, 1e-10, 2000, -1, use_graph)
    assert ok
    it2, res2, ok2 = tm.batch_cg_solve(members, 1e-10, 2000, -1, use_graph)
    assert ok2 and max(it2) == 0 and res2 == res
    for m in members:
        m["x"].zero_()
    members[1]["x"][2].fill_(0.5)       # one system starts elsewhere
    it3, res3, ok3 = tm.batch_cg_solve(members, 1e-10, 2000, -1, use_graph)
    assert ok3 and max(res3) <= 1e-10
    dims, U, bs = host_data[1]
    x = host(tm.spinor_export(members[1]["lat"], members[1]["x"][2]))
    rr = bs[2] - oracle.normal(dims, U, x, kappa, mu, THETA_AP)
    assert np.linalg.norm(rr) / np.linalg.norm(bs[2]) <= 1.05e-10


def test_batch_not_converged_reported():
    members, _, _, _ = batch_problem()
    it, res, ok = tm.batch_cg_solve(members, 1e-10, 3, -1, True)
    assert not ok and max(it) <= 3 * 4 and max(res) > 1e-10


def test_autotune_and_cache(tmp_path):
    dims = (8, 8, 8, 8)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, haar(dims, 551))
    cache = str(tmp_path / "tune.txt")
    sh, us = tm.autotune_mrhs(lat, G, 12, tm.F64, cache)
    assert 0 <= sh < len(tm.tmhop.SHAPES) and us > 0
    text = open(cache).read().split()
    assert text[1] == "8x8x8x8" and text[2] == "f64" and text[3] == "12" and int(text[4]) == sh
    lat2 = tm.Lattice(dims)
    sh2, us2 = tm.autotune_mrhs(lat2, tm.gauge_import(lat2, haar(dims, 551)), 12, tm.F64, cache)
    assert (sh2, us2) == (sh, float(text[5]))
    assert len(open(cache).read().strip().splitlines()) == 1


@pytest.mark.parametrize("use_graph", [False, True], ids=["eager", "graph"])
def test_batch_zero_source_nonzero_start(use_graph):
    """A system with b = 0 and a start vector that is not zero gets x = 0 and
    residual 0 without holding back the others (as tmh_cg_solve does), alone
    in a batch and beside other systems."""
    kappa, mu = 0.1632, mu_of(0.1632, 0.0013)
    dims = (4, 4, 4, 4)
    lat = tm.Lattice(dims)
    U = haar(dims, 25)
    G = tm.gauge_import(lat, U)
    # alone: one member, one system
    x = lat.new_spinors(1)
    x.fill_(1.0)
    b = lat.new_spinors(1)
    it, res, ok = tm.batch_cg_solve([dict(lat=lat, x=x, b=b, gauge=G, kappa=kappa, mu=mu, theta=THETA_AP)],
                                    1e-10, 100, -1, use_graph)
    assert ok and it == [0] and res == [0.0] and float(x.abs().max()) == 0.0
    # beside two systems with Gaussian sources, on a second lattice as well
    dims2 = (6, 8, 10, 4)
    lat2 = tm.Lattice(dims2)
    U2 = haar(dims2, 531)
    bs = [gauss(lat.Vh, 26), np.zeros((lat.Vh, 4, 3), np.complex128), gauss(lat.Vh, 27)]
    b3 = import_many(lat, bs)
    x3 = lat.new_spinors(3)
    x3[1].fill_(0.25)
    b2 = import_many(lat2, [gauss(lat2.Vh, 28)])
    x2 = lat2.new_spinors(1)
    members = [dict(lat=lat, x=x3, b=b3, gauge=G, kappa=kappa, mu=mu, theta=THETA_AP),
               dict(lat=lat2, x=x2, b=b2, gauge=tm.gauge_import(lat2, U2), kappa=kappa, mu=mu, theta=THETA_AP)]
    it, res, ok = tm.batch_cg_solve(members, 1e-10, 500, -1, use_graph)
    assert ok and it[1] == 0 and res[1] == 0.0 and float(x3[1].abs().max()) == 0.0
    assert max(it) < 500
    for r in (0, 2):
        xs = host(tm.spinor_export(lat, x3[r]))
        rr = bs[r] - oracle.normal(dims, U, xs, kappa, mu, THETA_AP)
        assert np.linalg.norm(rr) / np.linalg.norm(bs[r]) <= 1.05e-10, r


@pytest.mark.parametrize("prec", [tm.F64, tm.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("nrhs", [1, 4, 12])
@pytest.mark.parametrize("dims", [(6, 8, 10, 4), (8, 4, 16, 16)], ids=["6x8x10x4", "8x4x16x16"])
def test_hop_mrhs_mfma_matches_oracle_and_vector_path(dims, nrhs, prec):
    """The matrix-core shape against the oracle (1e-13 FP64, 1e-5 FP32) for
    1, 4 and 12 right-hand sides (a ragged group of 8 for 4 and 12, a ragged
    last tile on 6x8x10x4), and against the vector path of the same run."""
    kappa = 0.15
    U = haar(dims, 561)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U, prec)
    psis = [gauss(lat.Vh, 570 + r) for r in range(nrhs)]
    inp = import_many(lat, psis, prec)
    tol = 1e-13 if prec == tm.F64 else 1e-5
    for direction in ("eo", "oe"):
        out = lat.new_spinors(nrhs, prec)
        tm.hop_apply_mrhs(lat, direction, out, G, inp, kappa, TWIST, prec, tm.tmhop.MFMA)
        vec = lat.new_spinors(nrhs, prec)
        tm.hop_apply_mrhs(lat, direction, vec, G, inp, kappa, TWIST, prec, 0)
        for r in range(nrhs):
            ref = oracle.hop(dims, direction, U, psis[r], kappa, TWIST)
            got = host(tm.spinor_export(lat, out[r], prec))
            assert site_rel_err(got, ref) <= tol, (direction, r)
            assert site_rel_err(got, host(tm.spinor_export(lat, vec[r], prec))) <= tol, (direction, r)


@pytest.mark.parametrize("use_graph", [False, True], ids=["eager", "graph"])
def test_batch_cg_mfma_shape(use_graph):
    """The batched CG on the matrix-core shape (its fused epilogues: A^-1
    store, twist + norm, CG update) reaches the oracle-certified residual."""
    members, host_data, kappa, mu = batch_problem()
    it, res, ok = tm.batch_cg_solve(members, 1e-10, 2000, tm.tmhop.MFMA, use_graph)
    assert ok and max(res) <= 1e-10
    for m, (dims, U, bs) in zip(members, host_data):
        for r, b in enumerate(bs):
            x = host(tm.spinor_export(m["lat"], m["x"][r]))
            rr = b - oracle.normal(dims, U, x, kappa, mu, THETA_AP)
            assert np.linalg.norm(rr) / np.linalg.norm(b) <= 1.05e-10, (dims, r)


@pytest.mark.parametrize("prec", [tm.F64, tm.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape", list(tm.tmhop.TMARCH_SHAPES), ids=["tmarch", "tmarch-pipe", "tmarch4", "tmarch4-lds"])
@pytest.mark.parametrize("dims", [(32, 16, 16, 16), (64, 8, 8, 16)], ids=["32x16x16x16", "64x8x8x16"])
def test_hop_mrhs_tmarch_several_steps(dims, shape, prec):
    """Lattices big enough for the t-march to walk several time-slices per
    workgroup with 12 right-hand sides (4 and 2 steps): the register ring
    carries the time neighbours across steps and range boundaries; against
    the oracle, and within 1e-14 per site of the one-site-per-lane shape in
    FP64 (the same sums; the compiler may fuse their multiply-adds
    differently in the two kernels)."""
    kappa, nrhs = 0.15, 12
    U = haar(dims, 581)
    lat = tm.Lattice(dims)
    G = tm.gauge_import(lat, U, prec)
    psis = [gauss(lat.Vh, 590 + r) for r in range(nrhs)]
    inp = import_many(lat, psis, prec)
    tol = 1e-13 if prec == tm.F64 else 1e-5
    for direction in ("eo", "oe"):
        out = lat.new_spinors(nrhs, prec)
        tm.hop_apply_mrhs(lat, direction, out, G, inp, kappa, TWIST, prec, shape)
        base = lat.new_spinors(nrhs, prec)
        tm.hop_apply_mrhs(lat, direction, base, G, inp, kappa, TWIST, prec, 0)
        for r in (0, 5, 11):
            ref = oracle.hop(dims, direction, U, psis[r], kappa, TWIST)
            got = host(tm.spinor_export(lat, out[r], prec))
            assert site_rel_err(got, ref) <= tol, (direction, r)
            if prec == tm.F64:
                assert site_rel_err(got, host(tm.spinor_export(lat, base[r], prec))) <= 1e-14, (direction, r)


@pytest.mark.parametrize("use_graph", [False, True], ids=["eager", "graph"])
@pytest.mark.parametrize("shape", list(tm.tmhop.TMARCH_SHAPES), ids=["tmarch", "tmarch-pipe", "tmarch4", "tmarch4-lds"])
def test_batch_cg_tmarch_shapes(shape, use_graph):
    """The batched CG on the t-march shapes (fused A^-1 store, twist + norm
    with one partial per system and slice tile, CG update) over two
    lattices, one walking two time-slices per workgroup: certified by the
    oracle and iterating like the single-system CG."""
    kappa, mu = 0.1632, mu_of(0.1632, 0.0013)
    members, host_data = [], []
    for dims, nrhs, seed in (((32, 16, 16, 16), 4, 601), ((8, 8, 8, 8), 3, 611)):
        lat = tm.Lattice(dims)
        U = haar(dims, seed)
        bs = [gauss(lat.Vh, seed + 1 + r) for r in range(nrhs)]
        members.append(dict(lat=lat, x=lat.new_spinors(nrhs), b=import_many(lat, bs),
                            gauge=tm.gauge_import(lat, U), kappa=kappa, mu=mu, theta=THETA_AP))
        host_data.append((dims, U, bs))
    it, res, ok = tm.batch_cg_solve(members, 1e-10, 2000, shape, use_graph)
    assert ok and max(res) <= 1e-10
    k = 0
    for m, (dims, U, bs) in zip(members, host_data):
        for r, b in enumerate(bs):
            x = host(tm.spinor_export(m["lat"], m["x"][r]))
            rr = b - oracle.normal(dims, U, x, kappa, mu, THETA_AP)
            assert np.linalg.norm(rr) / np.linalg.norm(b) <= 1.05e-10, (dims, r)
            if r == 0:
                x1 = m["lat"].new_spinor()
                it1, _, ok1 = tm.cg_solve(m["lat"], x1, m["b"][r].contiguous(), m["gauge"], kappa, mu,
                                          THETA_AP, 1e-10, 2000)
                assert ok1 and abs(it1 - it[k]) <= 2
            k += 1


@pytest.mark.slow
def test_hop_mrhs_full_size_32x32x32x64():
    """The benchmark lattice with 12 right-hand sides, in the shapes the
    batched CG and the autotuner pick there (the LDS-staged t-march in FP64
    and FP32, the pipelined t-march): every boundary time-slice and 5,000
    random sites of 3 of the right-hand sides against the oracle, and all
    sites and right-hand sides against the one-site-per-lane shape."""
    dims, kappa, nrhs = (64, 32, 32, 32), 0.1632, 12
    U = haar(dims, 951)
    lat = tm.Lattice(dims)
    Vh = lat.Vh
    psis = [gauss(Vh, 960 + r) for r in range(nrhs)]
    g = np.random.default_rng(97)
    slab = dims[1] * dims[2] * dims[3] // 2
    sites = np.unique(np.concatenate([np.arange(slab), np.arange(Vh - slab, Vh), g.integers(0, Vh, 5000)]))
    for prec, tol, same in ((tm.F64, 1e-13, 1e-14), (tm.F32, 1e-5, 1e-6)):
        G = tm.gauge_import(lat, U, prec)
        inp = import_many(lat, psis, prec)
        base = lat.new_spinors(nrhs, prec)
        tm.hop_apply_mrhs(lat, "eo", base, G, inp, kappa, THETA_AP, prec, "256x1")
        for shape in ("64x4/tmarch-lds", "256x1/tmarch-pipe"):
            out = lat.new_spinors(nrhs, prec)
            tm.hop_apply_mrhs(lat, "eo", out, G, inp, kappa, THETA_AP, prec, shape)
            for r in (0, 5, 11):
                src = psis[r] if prec == tm.F64 else round_f32(psis[r])
                ref = oracle.hop_sites(dims, "eo", sites, U if prec == tm.F64 else round_f32(U), src, kappa,
                                       THETA_AP)
                got = host(tm.spinor_export(lat, out[r], prec))
                assert site_rel_err(got[sites], ref) <= tol, (prec, shape, r)
            for r in range(nrhs):
                assert site_rel_err(host(tm.spinor_export(lat, out[r], prec)),
                                    host(tm.spinor_export(lat, base[r], prec))) <= same, (prec, shape, r)
            del out
        del G, inp, base


@pytest.mark.slow
def test_batch_cg_full_size_32x32x32x64():
    """The batched CG with 12 right-hand sides on the benchmark lattice, on
    the LDS-staged t-march shape the batch workload picks: every system
    converges to 1e-10 by the solver's own FP64 true residual, two of them
    are certified by the oracle's operator, and they agree with the
    single-system CG."""
    dims, kappa, nrhs = (64, 32, 32, 32), 0.1632, 12
    mu = mu_of(kappa, 0.0013)
    U = haar(dims, 971)
    lat = tm.Lattice(dims)
    bs = [gauss(lat.Vh, 980 + r) for r in range(nrhs)]
    G = tm.gauge_import(lat, U)
    m = dict(lat=lat, x=lat.new_spinors(nrhs), b=import_many(lat, bs), gauge=G, kappa=kappa, mu=mu, theta=THETA_AP)
    it, res, ok = tm.batch_cg_solve([m], 1e-10, 2000, "64x4/tmarch-lds", True)
    assert ok and max(res) <= 1e-10
    for r in (0, 7):
        x = host(tm.spinor_export(lat, m["x"][r]))
        rr = bs[r] - oracle.normal(dims, U, x, kappa, mu, THETA_AP)
        assert np.linalg.norm(rr) / np.linalg.norm(bs[r]) <= 1.05e-10, r
    x1 = lat.new_spinor()
    it1, _, ok1 = tm.cg_solve(lat, x1, m["b"][3].contiguous(), G, kappa, mu, THETA_AP, 1e-10, 2000)
    assert ok1 and abs(it1 - it[3]) <= 2
    d = host(tm.spinor_export(lat, x1)) - host(tm.spinor_export(lat, m["x"][3]))
    assert np.linalg.norm(d) / np.linalg.norm(host(tm.spinor_export(lat, x1))) <= 1e-8
