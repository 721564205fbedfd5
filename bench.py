#!/usr/bin/env python3
"""Benchmark of the hopping-matrix hot path on one MI355X; prints one JSON line.

Workload (default ``qtm32``): 32^3x64 lattice, Haar-random SU(3) links, a
Gaussian odd source, kappa = 0.1632, 2 kappa mu = 0.0013, antiperiodic time.
One step = one complete FP64 CG solve on Qhat^dagger Qhat to a 1e-10 true
relative residual (every hopping-matrix and twisted-mass application, BLAS-1
update and reduction of the path), with the inputs resident in HBM.

value = Dslash GFlop/s over the timed steps: 1320 flop per output site per
hopping-matrix application, times the applications the solves made, over the
wall time of the steps.  The roofline entry is for the dominant kernel, the
FP64 hopping matrix storing A^-1 H_eo p (1536 algorithmic bytes per site),
timed live with HIP events on the stream it runs on.  Beside it the same
system is solved by the mixed-precision (FP32 inner) defect-correction CG,
with 9-entry and with two-row FP32 links, by the same with FP16 storage in
the inner solve, and by FP64 CG on two-row FP64 links (the third row of each
SU(3) link rebuilt in the kernel); the CPU oracle is timed on a bounded
sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Dslash GFlop/s + % HBM roofline at 32^3x64; mixed vs FP64 CG time to 1e-10"
FLOP_PER_SITE = 1320
PREC_NAME = {0: "fp64", 1: "mixed fp32", 2: "fp64 two-row links", 3: "mixed fp32 two-row links",
             4: "mixed fp16 storage", 5: "mixed fp16 storage two-row links"}
BYTES_PER_SITE_F64 = 1536          # 8 links x 144 B + input spinor 192 B + output 192 B
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hop_f64_32x32x32x64_traffic.json")  # 32^3x64 only

WORKLOADS = {
    "qtm32": dict(dims=(64, 32, 32, 32), kappa=0.1632, mt=0.0013, seed=2, links="haar",
                  label="Qtm + FP64 CG to 1e-10 on 32^3x64, Haar SU(3) links, "
                        "kappa=0.1632, 2*kappa*mu=0.0013, antiperiodic time"),
    # the mixed-precision workload: smoothed links U = exp(i 0.3 H); the
    # paper's 48^3x96 inversion fixes no kappa or mu, the 32^3x64 values are reused
    "mixed48": dict(dims=(96, 48, 48, 48), kappa=0.1632, mt=0.0013, seed=3, links="smooth",
                    label="FP64 CG vs defect-correction CG (FP32 or FP16-storage inner) to 1e-10 "
                          "on 48^3x96, links exp(0.3 i H), kappa=0.1632, 2*kappa*mu=0.0013, "
                          "antiperiodic time"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(n_sites):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None if absent or taken on other code."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_1311_4521_amd.rocprof_summary import hop_source_hash
    if t.get("source_hash") != hop_source_hash() or t.get("sites") != n_sites:
        return None
    return round(t.get("bytes_per_launch"), 0)


def cpu_baseline(dims, U, psi, kappa, theta, budget_s, cg=None):
    import numpy as np

    import oracle
    Vh = len(psi)
    t0 = time.perf_counter()
    oracle.hop(dims, "eo", U, psi, kappa, theta)
    one = time.perf_counter() - t0
    reps = max(1, int(budget_s / max(one, 1e-9)))
    per = []
    for _ in range(reps):
        t1 = time.perf_counter()
        oracle.hop(dims, "eo", U, psi, kappa, theta)
        per.append(time.perf_counter() - t1)
    dt = sum(per)
    cores = oracle.num_threads()
    # the same sample on one thread, bounded to a few applications
    oracle.set_num_threads(1)
    try:
        reps1 = max(3, min(reps, int(0.25 * budget_s / max(one * cores, 1e-9))))
        t0 = time.perf_counter()
        for _ in range(reps1):
            oracle.hop(dims, "eo", U, psi, kappa, theta)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    out = {
        "value": round(FLOP_PER_SITE * Vh * reps / dt / 1e9, 3),
        "unit": "GFlop/s",
        "cores": cores,
        "host_cpus": os.cpu_count(),
        "kind": "oracle",
        "sample": f"{reps} oracle D_eo applications on the {'x'.join(map(str, dims))} fields "
                  f"({Vh} output sites each, {dt:.1f} s)",
        "median_ms_per_application": round(1e3 * float(np.median(per)), 2),
        "min_ms_per_application": round(1e3 * min(per), 2),
        "value_1_thread": round(FLOP_PER_SITE * Vh * reps1 / dt1 / 1e9, 3),
        "sample_1_thread": f"{reps1} applications on one thread ({dt1:.1f} s)",
    }
    if cg is not None:
        # one full oracle CG of the benchmark system on all threads, and its
        # solution against the GPU's FP64 one (both at true residual 1e-10)
        mu, x_gpu = cg
        t0 = time.perf_counter()
        x, it, res, ok = oracle.cg(dims, U, psi, kappa, mu, theta, 1e-10, 20000)
        dtc = time.perf_counter() - t0
        out["cg"] = {"seconds": round(dtc, 2), "iterations": it, "true_rel_res": res, "converged": ok,
                     "rel_diff_vs_gpu_fp64_solution":
                         float(np.linalg.norm(x - x_gpu) / np.linalg.norm(x))}
    return out


def hop_standalone(tm, lat, G, x, kappa, mu, theta, warm=10, reps=100):
    """Single hopping-matrix applications outside the solver: D_eo and D_oe
    on the resident FP64 fields, and one Q-hat+ application; each launch
    timed on its own with HIP events on the library's stream.  Median and
    minimum in us, with the algorithmic bandwidth at each."""
    import torch
    Vh = lat.Vh
    out = lat.new_spinor()
    res = {}

    def stats(us, nbytes):
        us = sorted(us)
        med = us[len(us) // 2] if len(us) % 2 else 0.5 * (us[len(us) // 2 - 1] + us[len(us) // 2])
        d = {"median_us": round(med, 2), "min_us": round(us[0], 2)}
        if nbytes:
            d["median_GBs"] = round(nbytes / (med * 1e-6) / 1e9, 1)
            d["min_GBs"] = round(nbytes / (us[0] * 1e-6) / 1e9, 1)
        return d

    def timed(fn):
        for _ in range(warm):
            fn()
        evs = [_events() for _ in range(reps)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return [a.elapsed_time(b) * 1e3 for a, b in evs]

    for d in ("eo", "oe"):
        res["hop_" + d] = stats(timed(lambda: tm.hop_apply(lat, d, out, G, x, kappa, theta)),
                                BYTES_PER_SITE_F64 * Vh)
    q = lat.new_spinor()
    res["qtm_plus"] = stats(timed(lambda: tm.qtm_apply(lat, q, G, x, kappa, mu, theta, +1)), None)
    res["timing"] = f"{warm} untimed, then {reps} applications each timed with HIP events"
    del out, q
    return res


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time_us(fn, reps=10, warm=2):
    import torch
    for _ in range(warm):
        fn()
    a, b = _events()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e3 / reps


COPY_BYTES = 805306368  # the streaming copy the counter summaries check against


def copy_reference(lat):
    """Streaming copies of COPY_BYTES (the achievable-bandwidth reference and
    the known-size kernel of the counter runs); returns GB/s of the last."""
    import torch

    from paper_1311_4521_amd import tmhop
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        tmhop.stream_copy(lat, dst, src)
    us = _time_us(lambda: tmhop.stream_copy(lat, dst, src), reps=3, warm=0)
    return round(2 * COPY_BYTES / (us * 1e-6) / 1e9, 1)


def run_batch(args):
    """12 Gaussian right-hand sides on each of 16^3x32, 24^3x48 and 32^3x64
    (Haar links): one batched CG (one launch per operator step for all 36
    systems, HIP-graph replay, autotuned tile shape) against the 36 solves
    one after another."""
    import numpy as np
    import torch

    import fieldgen
    import paper_1311_4521_amd as tm

    torch.cuda.set_device(0)
    kappa, mt, nrhs = 0.1632, 0.0013, 12
    mu = mt / (2 * kappa)
    theta = (1.0, 0.0, 0.0, 0.0)
    seed = fieldgen.SEEDS["batch"]
    members = []
    for k, dims in enumerate([(64, 32, 32, 32), (48, 24, 24, 24), (32, 16, 16, 16)]):
        log(f"batch member {dims}: generating links and {nrhs} sources")
        lat = tm.Lattice(dims, 0)
        G = tm.gauge_import(lat, fieldgen.gauge_haar(dims, seed + 10 * k))
        B = lat.new_spinors(nrhs)
        for r in range(nrhs):
            tm.spinor_import(lat, fieldgen.spinor_gauss(lat.Vh, 1000 * (k + 1) + r), out=B[r])
        members.append(dict(lat=lat, x=lat.new_spinors(nrhs), b=B, gauge=G, kappa=kappa, mu=mu,
                            theta=theta))
    big = members[0]
    copy_gbs = copy_reference(big["lat"])
    names = {v: k for k, v in tm.tmhop.SHAPES.items()}
    hop_shape, tuned_us = tm.autotune_mrhs(big["lat"], big["gauge"], nrhs, tm.F64, args.tune_cache)
    log(f"autotuned tile shape {names[hop_shape]}: {tuned_us:.1f} us per 12-RHS hop at 32^3x64")
    lat, G = big["lat"], big["gauge"]
    Vh = lat.Vh
    X1, Y1 = lat.new_spinor(), lat.new_spinor()
    single_us = _time_us(lambda: tm.hop_apply(lat, "eo", Y1, G, X1, kappa, theta))
    Xm, Ym = lat.new_spinors(nrhs), lat.new_spinors(nrhs)
    multi_us = _time_us(lambda: tm.hop_apply_mrhs(lat, "eo", Ym, G, Xm, kappa, theta, tm.F64, hop_shape))
    # the plain hop ranks the shapes; the batched CG, whose last hop of an
    # iteration also carries the CG update of every right-hand side, is
    # timed for the three fastest and runs with the best of them
    hop_us = {sh: _time_us(lambda sh=sh: tm.hop_apply_mrhs(lat, "eo", Ym, G, Xm, kappa, theta, tm.F64, sh),
                           reps=3, warm=1) for sh in tm.tmhop.SHAPES.values()}
    del Xm, Ym
    # the same in FP32: every shape, the matrix-core one among them
    G32 = tm.gauge_import(lat, fieldgen.gauge_haar(lat.dims, seed), tm.F32)
    Xs, Ys = lat.new_spinors(nrhs, tm.F32), lat.new_spinors(nrhs, tm.F32)
    Xs.normal_()
    hop_us32 = {sh: _time_us(lambda sh=sh: tm.hop_apply_mrhs(lat, "eo", Ys, G32, Xs, kappa, theta, tm.F32, sh),
                             reps=3, warm=1) for sh in tm.tmhop.SHAPES.values()}
    del G32, Xs, Ys
    mfma = {}
    for key, tab in (("f64", hop_us), ("f32", hop_us32)):
        vec = {k: v for k, v in tab.items() if k != tm.tmhop.MFMA}
        best = min(vec, key=vec.get)
        mfma[key] = {"mfma_us": round(tab[tm.tmhop.MFMA], 1), "best_vector_us": round(vec[best], 1),
                     "best_vector_shape": names[best],
                     "mfma_over_vector": round(tab[tm.tmhop.MFMA] / vec[best], 3)}
    log(f"12-RHS hop at 32^3x64, matrix cores against the best vector shape: {mfma}")
    mrhs_bytes = (1152 + nrhs * 384) * Vh

    def batched(sh):
        for m in members:
            m["x"].zero_()
        return tm.batch_cg_solve(members, 1e-10, 5000, sh, True)

    cg_ms = {}
    for sh in sorted(hop_us, key=hop_us.get)[:3]:
        batched(sh)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batched(sh)
        torch.cuda.synchronize()
        cg_ms[sh] = 1e3 * (time.perf_counter() - t0)
    shape = min(cg_ms, key=cg_ms.get)
    shape_name = names[shape]
    log(f"batched CG per shape (ms): {({names[k]: round(v, 1) for k, v in cg_ms.items()})}; using {shape_name}")

    it, res, ok = batched(shape)
    torch.cuda.synchronize()
    tb = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        it, res, ok = batched(shape)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        if not ok:
            raise SystemExit("batched CG did not converge")
    log(f"batched: {1e3 * min(tb):.1f} ms for {sum(m['b'].shape[0] for m in members)} systems")
    # the same systems one after another
    seq_it = []
    x = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m in members:
        x = m["lat"].new_spinor()
        for r in range(nrhs):
            x.zero_()
            i1, r1, ok1 = tm.cg_solve(m["lat"], x, m["b"][r], m["gauge"], kappa, mu, theta, 1e-10, 5000)
            seq_it.append(i1)
            if not ok1:
                raise SystemExit("sequential CG did not converge")
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    log(f"sequential: {1e3 * t_seq:.1f} ms")
    t_batch = min(tb)
    line = {
        "metric": "batched CG time to 1e-10, 12 RHS on each of 16^3x32, 24^3x48, 32^3x64, "
                  "vs the 36 solves one after another",
        "value": round(1e3 * t_batch, 2), "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(1e3 * t_batch, 2), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch: 3 Haar lattices x 12 Gaussian RHS, kappa=0.1632, "
                               "2*kappa*mu=0.0013, antiperiodic time", "tile_shape": shape_name,
                   "hop_tile_shape": names[hop_shape],
                   "batched_cg_ms_by_shape": {names[k]: round(v, 1) for k, v in cg_ms.items()}},
        "sequential_ms": round(1e3 * t_seq, 2),
        "copy_GBs": copy_gbs,
        "speedup_vs_sequential": round(t_seq / t_batch, 3),
        "iterations": {"batched_max": max(it), "sequential_max": max(seq_it)},
        "max_true_rel_res": max(res),
        "mrhs_hop_32x32x32x64": {"nrhs": nrhs, "us": round(multi_us, 1),
                                 "us_per_rhs": round(multi_us / nrhs, 2),
                                 "single_rhs_us": round(single_us, 1),
                                 "speedup_per_rhs": round(single_us * nrhs / multi_us, 3),
                                 "GBs_algorithmic": round(mrhs_bytes / (multi_us * 1e-6) / 1e9, 1),
                                 "bytes_per_site": 1152 + nrhs * 384,
                                 "GFlops": round(1320 * nrhs * Vh / (multi_us * 1e-6) / 1e9, 1),
                                 "us_by_shape_f64": {names[k]: round(v, 1) for k, v in hop_us.items()},
                                 "us_by_shape_f32": {names[k]: round(v, 1) for k, v in hop_us32.items()},
                                 "mfma": mfma},
    }
    print(json.dumps(line), flush=True)


def run_adjoint(args):
    """24^3x48 Haar links, Gaussian chi and psi: the su(3) force of
    Re<chi, Qhat psi> (two hops + two force kernels) and one forward +
    backward of the autograd function (psi and link gradients)."""
    import numpy as np
    import torch

    import fieldgen
    import paper_1311_4521_amd as tm
    from paper_1311_4521_amd import autograd as tag

    torch.cuda.set_device(0)
    dims, kappa, mt = (48, 24, 24, 24), 0.1632, 0.0013
    mu = mt / (2 * kappa)
    theta = (1.0, 0.0, 0.0, 0.0)
    seed = fieldgen.SEEDS["adjoint24"]
    U = fieldgen.gauge_haar(dims, seed)
    lat = tm.Lattice(dims, 0)
    Vh = lat.Vh
    chi = fieldgen.spinor_gauss(Vh, 100 + seed)
    psi = fieldgen.spinor_gauss(Vh, 200 + seed)
    G = tm.gauge_import(lat, U)
    tc, tp = tm.spinor_import(lat, chi), tm.spinor_import(lat, psi)
    F = lat.new_gauge(zero=True)
    copy_gbs = copy_reference(lat)
    force_us = _time_us(lambda: tm.hop_force(lat, "eo", F, G, tc, tp, kappa, theta))
    qforce_us = _time_us(lambda: tm.qtm_force(lat, F, G, tc, tp, kappa, mu, theta))
    Ut = torch.from_numpy(U).cuda().requires_grad_()
    pt = torch.from_numpy(psi).cuda().requires_grad_()
    ct = torch.from_numpy(chi).cuda()

    def fb():
        Ut.grad = None
        pt.grad = None
        L = tag.qtm_bilinear(lat, ct, pt, Ut, kappa, mu, theta)
        L.backward()

    ag_us = _time_us(fb, reps=5, warm=1)
    V = 2 * Vh
    fbytes = 1920 * V
    line = {
        "metric": "gauge-link force of Re<chi, Qhat psi> at 24^3x48",
        "value": round(qforce_us / 1e3, 4), "unit": "ms", "n_gpus": 1, "steps": 10, "warmup": 2,
        "ms_per_step": round(qforce_us / 1e3, 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "adjoint: 24^3x48 Haar links, Gaussian chi and psi, kappa=0.1632, "
                               "2*kappa*mu=0.0013"},
        "hop_force_kernel": {"us": round(force_us, 1), "bytes_per_site": 1920,
                             "GBs_algorithmic": round(fbytes / (force_us * 1e-6) / 1e9, 1),
                             "frac_of_8TBs": round(fbytes / (force_us * 1e-6) / 8e12, 4)},
        "qtm_force_us": round(qforce_us, 1),
        "copy_GBs": copy_gbs,
        "autograd_forward_backward_ms": round(ag_us / 1e3, 3),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="qtm32", choices=sorted(WORKLOADS) + ["batch", "adjoint24"])
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (batch workload)")
    ap.add_argument("--xgroup", type=int, default=None,
                    help="fix the hop traversal x-group instead of autotuning it (profiling runs)")
    ap.add_argument("--mixed-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-standalone", action="store_true",
                    help="skip the standalone hop/Qtm timings (profiling runs: they launch the same kernels)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the lattice would be split along T, then Z, one process per GPU)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "adjoint24":
        return run_adjoint(args)

    import numpy as np
    import torch

    import fieldgen
    import paper_1311_4521_amd as tm
    from paper_1311_4521_amd import tmhop

    w = WORKLOADS[args.workload]
    dims, kappa, mt = w["dims"], w["kappa"], w["mt"]
    mu = mt / (2 * kappa)
    theta = (1.0, 0.0, 0.0, 0.0)
    torch.cuda.set_device(0)

    log(f"generating fields {dims} (seed {w['seed']}, {w['links']} links)")
    if w["links"] == "haar":
        U = fieldgen.gauge_haar(dims, w["seed"])
    else:
        U = fieldgen.gauge_smooth(dims, w["seed"], 0.3)
    Vh = int(np.prod(dims)) // 2
    b = fieldgen.spinor_gauss(Vh, 100 + w["seed"])

    lat = tm.Lattice(dims, 0)
    G = tm.gauge_import(lat, U)
    tb = tm.spinor_import(lat, b)
    x = lat.new_spinor()
    by_code = {}
    if args.xgroup is None:
        # every storage code the solves below launch gets its own traversal
        for prec in (tm.F32, tm.F32_R12, tm.F64_R12, tm.F16, tm.F16_R12):
            Gp = tm.gauge_import(lat, U, prec)
            by_code[tmhop.PREC_NAMES[prec]] = tm.autotune_hop(lat, Gp, prec)[0]
            del Gp
        xgroup, tuned_us = tm.autotune_hop(lat, G, tm.F64)
        by_code["f64"] = xgroup
        log(f"fields resident on the device; hop traversal x-group {xgroup} ({tuned_us:.1f} us, autotuned); "
            f"per storage code {by_code}")
    else:
        lat.traversal = xgroup = args.xgroup
        log(f"fields resident on the device; hop traversal x-group {xgroup} (fixed)")

    def solve(inner):
        x.zero_()
        return tm.cg_solve(lat, x, tb, G, kappa, mu, theta, 1e-10, 20000, inner)

    for k in range(args.warmup):
        it, res, ok = solve(tm.F64)
        log(f"warmup {k}: {it} iterations, true residual {res:.3e}")

    # ---- timed region: K full FP64 solves
    tmhop.profile_enable(lat, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for k in range(args.steps):
        it, res, ok = solve(tm.F64)
        iters.append(it)
        if not ok:
            raise SystemExit(f"FP64 CG did not converge (residual {res})")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    counts = [tmhop.profile_read(lat, k) for k in range(tmhop.PROFILE_KINDS)]
    tmhop.profile_enable(lat, False)
    log(f"timed {args.steps} FP64 solves: {dt * 1e3 / args.steps:.2f} ms each, {iters[0]} iterations")
    x64 = x.clone()
    res64 = res

    n_hops = sum(c[0] for c in counts)
    value = FLOP_PER_SITE * Vh * n_hops / dt / 1e9
    n0, ms0 = counts[tmhop.profile_kind(tm.F64, 0)]
    hop_us = ms0 * 1e3 / n0
    achieved = BYTES_PER_SITE_F64 * Vh / (hop_us * 1e-6) / 1e9
    per_kind = {}
    names = tmhop.PROFILE_NAMES
    for k, (n, ms) in enumerate(counts):
        if n:
            per_kind[names[k]] = {"launches": n, "avg_us": round(ms * 1e3 / n, 2)}

    # ---- achievable-bandwidth reference: streaming copy of the hop's bytes
    half = BYTES_PER_SITE_F64 * Vh // 2 // 16 * 16
    src = torch.empty(half // 8, dtype=torch.float64, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        tmhop.stream_copy(lat, dst, src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(20):
        tmhop.stream_copy(lat, dst, src)
    ev1.record()
    torch.cuda.synchronize()
    copy_us = ev0.elapsed_time(ev1) * 1e3 / 20
    copy_gbs = 2 * half / (copy_us * 1e-6) / 1e9
    del src, dst
    log(f"streaming copy reference: {copy_gbs:.0f} GB/s ({2 * half} bytes moved per copy)")

    # ---- the other solvers of the same system beside it: FP32-inner defect
    # correction (9-entry and two-row FP32 links) and FP64 on two-row links
    def time_solve(inner, reps):
        times = []
        for k in range(1 + reps):
            tmhop.profile_enable(lat, True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            it, res, ok = solve(inner)
            torch.cuda.synchronize()
            if not ok:
                raise SystemExit(f"CG ({PREC_NAME[inner]}) did not converge (residual {res})")
            if k > 0:
                times.append(time.perf_counter() - t1)
        kinds = {}
        for kk in range(tmhop.PROFILE_KINDS):
            n, ms = tmhop.profile_read(lat, kk)
            if n:
                kinds[tmhop.PROFILE_NAMES[kk]] = {"launches": n, "avg_us": round(ms * 1e3 / n, 2)}
        tmhop.profile_enable(lat, False)
        d = (x - x64).double()
        ms = 1e3 * sum(times) / len(times) if times else None
        log(f"{PREC_NAME[inner]} solve: {ms} ms, {it} (inner) iterations, true residual {res:.3e}")
        return {"ms": round(ms, 3) if ms else None, "iterations": it, "true_rel_res": res,
                "rel_diff_vs_fp64_solution": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(x64)),
                "speedup_vs_fp64": round(fp64_ms / ms, 3) if ms else None, "kernels": kinds}

    fp64_ms = dt * 1e3 / args.steps
    mixed = time_solve(tm.F32, args.mixed_steps)
    mixed_r12 = time_solve(tm.F32_R12, args.mixed_steps)
    fp64_r12 = time_solve(tm.F64_R12, args.mixed_steps)
    mixed_f16 = time_solve(tm.F16, args.mixed_steps)
    mixed_f16_r12 = time_solve(tm.F16_R12, args.mixed_steps)

    standalone = None
    if not args.no_standalone:
        log("standalone hop and Qtm applications")
        standalone = hop_standalone(tm, lat, G, tb, kappa, mu, theta)
    traffic = measured_traffic(Vh)
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFlop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fp64_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w["label"], "dims_TXYZ": list(dims), "kappa": kappa,
                   "two_kappa_mu": mt, "tol": 1e-10, "seed": w["seed"], "hop_traversal_xgroup": xgroup,
                   "hop_traversal_by_code": by_code or None},
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "kernel": "hop_kernel<double,0,0> (A^-1 H_eo store, 9-entry links)",
            "bytes_per_site": BYTES_PER_SITE_F64,
            "avg_us": round(hop_us, 2),
            "launches": n0,
            "copy_reference_GBs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
        },
        "hop_gflops": round(FLOP_PER_SITE * Vh / (hop_us * 1e-6) / 1e9, 1),
        "kernels": per_kind,
        "standalone": standalone,
        "cg_fp64": {"ms": round(fp64_ms, 3), "iterations": iters[0], "true_rel_res": res64},
        "cg_mixed_f32": mixed,
        "cg_mixed_f32_r12": mixed_r12,
        "cg_fp64_r12": fp64_r12,
        "cg_mixed_f16": mixed_f16,
        "cg_mixed_f16_r12": mixed_f16_r12,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        x_gpu = tm.spinor_export(lat, x64).cpu().numpy()
        line["cpu_baseline"] = cpu_baseline(dims, U, b, kappa, theta, args.cpu_seconds, cg=(mu, x_gpu))
    print(json.dumps(line), flush=True)
    lat.close()


if __name__ == "__main__":
    main()
