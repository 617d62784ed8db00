#!/usr/bin/env python3
"""Benchmark of the layered-media dyadic FMM on one MI355X.

Workload: three-layer medium (interfaces z = 0, -1.2; k = 1.2, 2.0, 1.5),
N = 1e6 points uniform in [-4,4]^2 slabs (40/30/30 %, 0.05 from interfaces),
targets = sources, one complex128 current vector, p = 12.  A step is one
evaluation A = G J (P2M, M2M, M2L, L2L, L2P and the near field) on the built
geometry (trees and M2L tables prebuilt, their time is reported separately
as build_s); inputs are resident in HBM before the timed region.

Prints one JSON line (rank 0).  Only one GPU is used: --gpus N with N > 1
exits with a message.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "targets/s, 3-layer dyadic FMM N=1M p=12 at rel err≤1e-6; batched/adjoint vs plain"
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 64 fp64 FMA/clk x 2 flop x 2.4 GHz (fp64 MFMA: same)
HBM_PEAK_GBS = 8000.0
# algorithmic work of the near-field kernels (see the kernel table of the design notes):
# free-space pair: distance, 1/r, e^{ikr} (one sincos) and the two coefficients per kernel
# evaluation (60), the a q + b R (R.q) dyadic form per ordered pair (40); when the targets
# are the sources one evaluation serves both orders of a pair of different leaves
P2P_FLOPS_PER_EVAL = 60
P2P_FLOPS_PER_APPLY = 40
P2P_FLOPS_PER_PAIR = P2P_FLOPS_PER_EVAL + P2P_FLOPS_PER_APPLY
# direct reaction pair, per quadrature node: Z = exp(i (k_z t + k'_z u)), J0..J2 of
# k_rho rho, and the five complex multiply-adds of the node's contribution
S2T_FLOPS_PER_NODE = 100

# HBM traffic of one k_m2l launch at the default workload (N=1e6, p=12,
# p_free=20), from rocprofv3 FETCH_SIZE / WRITE_SIZE per dispatch scaled by a
# plain 1 GiB device copy (FETCH_SIZE reads 0.5 KiB per KiB read: factor 2.0;
# WRITE_SIZE 1:1), averaged over the evaluation's two launches; see
# profiles/k_m2l_three_layer_1M_p12_pf20.md.  Valid only for the kernel and
# tile-order source it was measured on (digest below), the same launches per
# step and the same M2L work; otherwise reported as null.
K_M2L_TRAFFIC = {"digest": "ce9a57772387ed21", "launches_per_step": 2, "m2l_cmac_useful": 619120501668.0,
                 "fetch_bytes": 0.5 * (3.5078e7 + 2.0243e7) * 1024 * 2.0,
                 "write_bytes": 0.5 * (2.3779e7 + 2.1319e7) * 1024 * 1.0}


def m2l_source_digest():
    """Digest of the M2L GEMM kernel's source and of the host code that
    orders its tiles (both decide its memory traffic)."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2507_18491_amd", "csrc", "kernels.hip")).read()
    a = src.index("// ------------------------------------------------------------------ M2L")
    b = src.index("// LE_t[out][rhs] += sum")
    api = open(os.path.join(ROOT, "paper_2507_18491_amd", "csrc", "api.cpp")).read()
    c = api.index("static int make_schedule(lm_ctx* ctx, int n_rhs, long long budget, lm_ctx::TileSet& ts, long long* block_max) {")
    e = api.index("// complex numbers of the P2M partial expansions")
    return hashlib.sha256((src[a:b] + api[c:e]).encode()).hexdigest()[:16]


def host_cores():
    """Host threads for the CPU baseline: the CPUs this process may run on,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(d, k, x, J, n_total, budget_s=15.0, budget_1core_s=8.0):
    """The oracle (direct Sommerfeld sum) timed on the host cores on a
    bounded sample: 16 sampled targets against ns sampled sources, on every
    core of the host share and on one core; the rates are scaled to
    targets/s of the full N-source sum."""
    from oracle import oracle
    threads = host_cores()
    rng = np.random.default_rng(11)
    ti = rng.choice(x.shape[0], 16, replace=False)
    si = rng.choice(x.shape[0], 200, replace=False)
    t = time.time()
    oracle.direct(d, k, x[si], J[si], x[ti], n_threads=threads)
    dt = time.time() - t
    scale = max(1.0, min(50.0, budget_s / max(dt, 1e-3)))
    nt = 16
    ns = int(200 * scale)
    si = rng.choice(x.shape[0], ns, replace=False)
    t = time.time()
    oracle.direct(d, k, x[si], J[si], x[ti], n_threads=threads)
    dt = time.time() - t
    pairs = nt * ns
    rate = pairs / dt
    # one core: 4 targets against a source sample sized from the multi-core rate
    ns1 = max(20, int(budget_1core_s * rate / threads / 4))
    si1 = rng.choice(x.shape[0], ns1, replace=False)
    t = time.time()
    oracle.direct(d, k, x[si1], J[si1], x[ti[:4]], n_threads=1)
    dt1 = time.time() - t
    rate1 = 4 * ns1 / dt1
    return {"value": rate / n_total, "unit": "targets/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "value_1core": rate1 / n_total,
            "sample": "%d sampled targets x %d sampled sources (%d pairs) in %.1f s on %d threads; one core: "
                      "4 targets x %d sources in %.1f s; rates scaled to the full %d-source sum" % (
                          nt, ns, pairs, dt, threads, ns1, dt1, n_total)}


def uneven_geometries(args, torch, inputs, lmfmm):
    """32 clustered geometries of 5e3 .. 2e5 points built into one plan; one
    evaluation of all of them captured in a HIP graph and replayed."""
    d, k, xs, Js = inputs.uneven_geometries(32, seed=0)
    n = sum(x.shape[0] for x in xs)
    t0 = time.time()
    f = lmfmm.LayeredDyadicFMM(d, k, p=args.p, p_free=args.p_free).build_batch(xs)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    J = torch.tensor(np.concatenate(Js), device="cuda:0").reshape(1, n, 3)
    A = torch.empty((1, n, 3), dtype=torch.complex128, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        f.evaluate(J, out=A)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        f.evaluate(J, out=A)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    dt = (time.time() - t0) / args.steps
    f.close()
    print("uneven geometries: %d points in 32 geometries, %.1f ms per graph replay, build %.2f s" % (
        n, 1e3 * dt, build_s), file=sys.stderr, flush=True)
    return {"targets_per_s": n / dt, "n_points": n, "n_geometries": 32, "ms_per_step": 1e3 * dt,
            "build_s": build_s, "launch": "hip graph replay of one evaluation"}


def batched_rhs(args, torch, inputs, lmfmm, n=200000, n_rhs=64, p=13):
    """Many current vectors on one tree: the three-layer geometry at n points
    with n_rhs vectors in one call, against the same tree with one vector per
    call (targets x right-hand sides per second).  Reaction order 13: at this
    size order 12 leaves 1.5e-6 against the oracle, order 13 6.8e-7."""
    d, k, x, J = inputs.three_layer(n, seed=0, n_rhs=n_rhs)
    f = lmfmm.LayeredDyadicFMM(d, k, p=p, p_free=args.p_free).build(x)
    Jm = torch.tensor(J, device="cuda:0")
    A = torch.empty_like(Jm)
    f.evaluate(Jm, out=A)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 2))
    t0 = time.time()
    for _ in range(steps):
        f.evaluate(Jm, out=A)
    torch.cuda.synchronize()
    dt_b = (time.time() - t0) / steps
    J1 = Jm[0].contiguous()
    A1 = torch.empty_like(J1)
    f.evaluate(J1, out=A1)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        f.evaluate(J1, out=A1)
    torch.cuda.synchronize()
    dt_1 = (time.time() - t0) / args.steps
    f.close()
    print("batched: %d points x %d right-hand sides, %.1f ms per call (one vector: %.1f ms)" % (
        n, n_rhs, 1e3 * dt_b, 1e3 * dt_1), file=sys.stderr, flush=True)
    return {"n": n, "n_rhs": n_rhs, "p": p, "p_free": args.p_free, "ms_per_call": 1e3 * dt_b,
            "targets_rhs_per_s": n * n_rhs / dt_b,
            "plain_ms_per_call": 1e3 * dt_1, "plain_targets_per_s": n / dt_1,
            "vs_plain": (n * n_rhs / dt_b) / (n / dt_1)}


def coupled_dipole_solve(args, torch, inputs, lmfmm, n=1000000, n_rhs=1, tol=1e-6, restart=30):
    """Restarted GMRES for the coupled-dipole system (diag - G) X = B on a
    jittered lattice of about n points filling the three-layer slabs (small
    dielectric spheres, eps_r = 2.25), seeded excitations; the operator is the
    same FMM at the benchmark's orders.  Reports iterations, time per
    iteration, the share of the operator applications and the achieved
    bandwidth of the Krylov vector kernels."""
    d, k, x, dg, B = inputs.dipole_lattice(n, seed=0, n_rhs=n_rhs)
    t0 = time.time()
    f = lmfmm.LayeredDyadicFMM(d, k, p=args.p, p_free=args.p_free).build(x)
    build_s = time.time() - t0
    Dg = torch.tensor(dg, device="cuda:0")
    Bt = torch.tensor(B, device="cuda:0")
    f.evaluate(Bt)  # first evaluation: M2L tuning outside the timed solve
    torch.cuda.synchronize()
    t0 = time.time()
    X, info = f.solve(Dg, Bt, tol=tol, restart=restart, max_iter=500)
    torch.cuda.synchronize()
    wall = time.time() - t0
    f.close()
    npts = x.shape[0]
    kb = info["krylov_bytes"] / (1e-3 * info["ms_krylov"]) / 1e9 if info["ms_krylov"] > 0 else None
    print("solve: %d lattice points, %d rhs, %d iterations (%d cycles), relres %.2e, %.2f s (operator %.0f %%)" % (
        npts, n_rhs, info["iters"], info["cycles"], float(np.max(info["relres"])), wall,
        100.0 * info["ms_matvec"] / max(1e-9, info["ms_total"])), file=sys.stderr, flush=True)
    return {"workload": "coupled-dipole system (diag - G) X = B, jittered lattice in the three-layer slabs, "
                        "eps_r 2.25 spheres, seeded excitations",
            "n": npts, "n_rhs": n_rhs, "tol": tol, "restart": restart, "iters": info["iters"],
            "matvecs": info["matvecs"], "cycles": info["cycles"], "converged": info["converged"],
            "relres_max": float(np.max(info["relres"])), "s_total": wall, "build_s": build_s,
            "ms_per_iter": info["ms_total"] / max(1, info["iters"]),
            "operator_share": info["ms_matvec"] / max(1e-9, info["ms_total"]),
            "krylov_ms": info["ms_krylov"],
            "krylov_roofline": {"bound": "hbm", "achieved": kb, "peak": 8000.0, "unit": "GB/s",
                                "frac": None if kb is None else kb / 8000.0,
                                "bytes": info["krylov_bytes"]}}


def trees_roofline(st):
    """The octrees' records keyed and radix-sorted on the device at build
    time (HBM-bound): algorithmic bytes per record -- the key kernel reads
    the position and the id and writes key, payload and tree (44 B); each of
    the eight key passes reads the key for the histogram and moves the
    16-byte record once (40 B), each tree pass the same plus the tree index
    (44 B) -- over the device time of those kernels."""
    recs, ms = st["tree_records"], st["tree_sort_ms"]
    if recs <= 0 or ms <= 0:
        return None
    n_trees = st["n_free_inst"] + 2 * st["n_react_inst"]
    tree_passes = 0
    t = int(n_trees) - 1
    while t > 0:
        tree_passes += 1
        t >>= 8
    per_rec = 44.0 + 8 * 40.0 + tree_passes * 44.0
    a = recs * per_rec / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "records": recs, "trees": n_trees, "device_ms": ms, "bytes_per_record": per_rec,
            "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a / HBM_PEAK_GBS,
            "plan_ms": st["t_plan_ms"]}


def largest_config(args, torch, inputs, lmfmm, n=2000000, n_rhs=16):
    """The largest configuration: four layers (interfaces 0, -1, -2.5; k =
    1.0, 1.8, 2.4, 1.3), N = 2e6 points (half uniform, half in 20 Gaussian
    clusters), p = 16 (free part p = 20), 16 current vectors in one call and
    their adjoint; one warm-up, then one timed call each, with the M2L GEMM
    roofline of the timed forward call."""
    d, k, x, J = inputs.four_layer(n, seed=0, n_rhs=n_rhs)
    t0 = time.time()
    f = lmfmm.LayeredDyadicFMM(d, k, p=16, p_free=20, m2l_variant=0).build(x)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    st = f.stats()
    Jt = torch.tensor(J, device="cuda:0")
    del J
    A = torch.empty_like(Jt)
    f.evaluate(Jt, out=A)
    torch.cuda.synchronize()
    f.set_timing(True)
    t0 = time.time()
    f.evaluate(Jt, out=A)
    torch.cuda.synchronize()
    fwd_s = time.time() - t0
    kt = f.kernel_timings()
    f.set_timing(False)
    gA = torch.tensor(inputs.cotangent(n, n_rhs=n_rhs, seed=0), device="cuda:0")
    gJ = torch.empty_like(gA)
    f.evaluate_adjoint(gA, out=gJ)
    torch.cuda.synchronize()
    t0 = time.time()
    f.evaluate_adjoint(gA, out=gJ)
    torch.cuda.synchronize()
    adj_s = time.time() - t0
    f.close()
    gms, gl = kt["m2l_gemm"]
    ach = st["m2l_cmac_useful"] * 8.0 * n_rhs / (gms * 1e-3) / 1e12 if gms > 0 else None
    print("largest: 2e6 points, 4 layers, p=16, %d rhs: forward %.2f s, adjoint %.2f s, build %.1f s" % (
        n_rhs, fwd_s, adj_s, build_s), file=sys.stderr, flush=True)
    return {"workload": "four-layer dyadic FMM, N=2e6 (half uniform, half in 20 Gaussian clusters), p=16 "
                        "(free part 20), 16 complex128 current vectors and their adjoint",
            "n": n, "n_rhs": n_rhs, "build_s": build_s,
            "forward_s": fwd_s, "targets_rhs_per_s": n * n_rhs / fwd_s,
            "adjoint_s": adj_s, "adjoint_targets_rhs_per_s": n * n_rhs / adj_s,
            "roofline": {"bound": "mfma", "kernel": "k_m2l", "achieved": ach, "peak": FP64_VALU_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": None if ach is None else ach / FP64_VALU_PEAK_TFLOPS,
                         "launches": gl, "gemm_ms": gms}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1000000)
    ap.add_argument("--p", type=int, default=12)
    ap.add_argument("--p-free", type=int, default=20)
    ap.add_argument("--rhs", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-uneven", action="store_true", help="skip the 32 uneven geometries")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-vector batched evaluation")
    ap.add_argument("--no-solve", action="store_true", help="skip the iterative coupled-dipole solve")
    ap.add_argument("--no-magnetic", action="store_true", help="skip the magnetic-field evaluation")
    ap.add_argument("--no-selfconv", action="store_true", help="skip the p = 16 self-convergence check")
    ap.add_argument("--no-largest", action="store_true",
                    help="skip the four-layer 2e6-point p = 16 16-vector configuration")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint and source-gradient timings (profiling runs of the forward step)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB device buffer three times (a reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read_per_copy": src.numel() * 8,
                          "copy_calibration_bytes_written_per_copy": src.numel() * 8}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (got --gpus %d); the evaluation would shard "
              "by independent FMM instances, but no multi-GPU run is provided." % args.gpus, flush=True)
        sys.exit(2)
    import torch
    from paper_2507_18491_amd import inputs, lmfmm

    d, k, x, J = inputs.three_layer(args.n, seed=0, n_rhs=args.rhs)
    dev = torch.device("cuda:0")
    # the HIP runtime's one-time start in this process is not part of a build
    torch.zeros(1, device=dev)
    torch.cuda.synchronize()
    t0 = time.time()
    fmm = lmfmm.LayeredDyadicFMM(d, k, p=args.p, p_free=args.p_free, device=0).build(x)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    st = fmm.stats()
    print("built: %.2f s (plan %.0f ms with the octree sort %.1f ms on the device for %d records, tables %.0f ms), "
          "m2l pairs free %d react %d, cases %d" % (
              build_s, st["t_plan_ms"], st["tree_sort_ms"], st["tree_records"], st["t_tables_ms"],
              st["m2l_pairs_free"], st["m2l_pairs_react"], st["n_cases"]), file=sys.stderr, flush=True)
    Jt = torch.tensor(J, device=dev)
    A = torch.empty((args.rhs, args.n, 3), dtype=torch.complex128, device=dev)
    for _ in range(args.warmup):
        fmm.evaluate(Jt.reshape(args.rhs, args.n, 3), out=A)
    torch.cuda.synchronize()
    fmm.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        fmm.evaluate(Jt.reshape(args.rhs, args.n, 3), out=A)
    torch.cuda.synchronize()
    wall = time.time() - t0
    phases, ncalls = fmm.timings()
    ktim = fmm.kernel_timings()
    gemm_ms_total, gemm_launches = fmm.m2l_gemm_timing()
    m2l_var, m2l_ms = fmm.m2l_variants(args.rhs)
    fmm.set_timing(False)
    ms_per_step = 1000.0 * wall / args.steps
    value = args.n * args.rhs / (wall / args.steps)
    # roofline of the M2L GEMM kernel: algorithmic flops (8 real flops per
    # complex multiply-add actually needed, absent-source columns excluded;
    # reaction pairs as the even and odd blocks of the mirror-adapted tensor)
    # per launch over the kernel's average launch duration.  The same M2L in
    # the dense spin-basis form (three P x 3P products per reaction pair)
    # needs about twice the work: reported beside it as the dense-equivalent
    # rate.
    launches_per_step = gemm_launches / max(1, ncalls)
    launch_ms = gemm_ms_total / max(1, gemm_launches)
    m2l_flops = st["m2l_cmac_useful"] * 8.0 * args.rhs
    flops_per_launch = m2l_flops / max(1e-30, launches_per_step)
    achieved = flops_per_launch / (launch_ms * 1e-3) / 1e12
    dense_per_launch = st["m2l_cmac_dense"] * 8.0 * args.rhs / max(1e-30, launches_per_step)
    # executed MFMA work (three real products per complex step, padded 16 x 16
    # tiles and k chunks): the matrix cores' own rate
    exec_per_launch = st["m2l_flop_exec"] * args.rhs / max(1e-30, launches_per_step)
    achieved_exec = exec_per_launch / (launch_ms * 1e-3) / 1e12

    def kroof(name, bound, work_per_step, unit):
        ms, launches = ktim[name]
        if launches == 0 or ms <= 0:
            return None
        per_launch = work_per_step * ncalls / launches
        sec = ms * 1e-3 / launches
        if unit == "GB/s":
            a = per_launch / sec / 1e9
            pk = HBM_PEAK_GBS
        else:
            a = per_launch / sec / 1e12
            pk = FP64_VALU_PEAK_TFLOPS
        return {"bound": bound, "achieved": a, "peak": pk, "unit": unit, "frac": a / pk,
                "launch_ms": ms / launches, "launches_per_step": launches / max(1, ncalls),
                "work_per_launch": per_launch}

    kernels = {
        "k_m2l_reduce": kroof("m2l_reduce", "hbm", st["reduce_bytes"] * args.rhs, "GB/s"),
        "k_p2p": kroof("p2p", "alu", (st["p2p_kernel_evals"] * P2P_FLOPS_PER_EVAL
                                      + st["p2p_pairs"] * P2P_FLOPS_PER_APPLY) * args.rhs, "TFLOP/s"),
        # the direct pairs' integrals are formed once per group of up to 4 vectors
        "k_s2t": kroof("s2t", "alu", st["s2t_node_evals"] * S2T_FLOPS_PER_NODE * ((args.rhs + 3) // 4), "TFLOP/s"),
    }
    # whole path: the sum of each kernel's ideal time at its own peak over the
    # measured time of the step
    t_ideal = (m2l_flops + (st["p2p_kernel_evals"] * P2P_FLOPS_PER_EVAL + st["p2p_pairs"] * P2P_FLOPS_PER_APPLY) * args.rhs
               + st["s2t_node_evals"] * S2T_FLOPS_PER_NODE * ((args.rhs + 3) // 4)
               + (st["p2m_flops"] + st["m2m_flops"] + st["l2l_flops"] + st["l2p_flops"]) * args.rhs
               ) / (FP64_VALU_PEAK_TFLOPS * 1e12)
    t_ideal += (st["reduce_bytes"] * args.rhs
                + (st["me_bytes_per_rhs"] + 2 * st["le_bytes_per_rhs"]) * args.rhs
                + 2 * 48.0 * args.n * args.rhs) / (HBM_PEAK_GBS * 1e9)
    path = {"t_ideal_ms": 1e3 * t_ideal, "t_measured_ms": ms_per_step, "frac": 1e3 * t_ideal / ms_per_step,
            "rule": "sum over kernels of algorithmic flops / 78.6 TFLOP/s (M2L, near field at %d flops per "
                    "pair, the kernel's 60 counted once per evaluation, direct reaction pairs at %d flops per quadrature node, P2M/M2M/L2L/L2P at 8 flops "
                    "per complex multiply-add) plus bytes / 8 TB/s (M2L reduction, expansion clears, "
                    "reading J and writing A)" % (P2P_FLOPS_PER_PAIR, S2T_FLOPS_PER_NODE)}
    print("timed: %.1f ms/step, phases (ms/step): %s" % (
        ms_per_step, {a: round(b / max(1, ncalls), 2) for a, b in phases.items()}), file=sys.stderr, flush=True)

    # adjoint (gJ = G^H gA) and source-position gradient on the same build,
    # timed like the forward step (same number of steps, after one warm-up)
    adj_s = grad_s = None
    if not args.no_adjoint:
        gA = torch.tensor(inputs.cotangent(args.n, n_rhs=args.rhs, seed=0), device=dev).reshape(args.rhs, args.n, 3)
        gJ = torch.empty_like(A)
        fmm.evaluate_adjoint(gA, out=gJ)
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(args.steps):
            fmm.evaluate_adjoint(gA, out=gJ)
        torch.cuda.synchronize()
        adj_s = (time.time() - t0) / args.steps
        gX = torch.empty((args.n, 3), dtype=torch.float64, device=dev)
        fmm.grad_src_xyz(Jt.reshape(args.rhs, args.n, 3), gA, out=gX)
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(args.steps):
            fmm.grad_src_xyz(Jt.reshape(args.rhs, args.n, 3), gA, out=gX)
        torch.cuda.synchronize()
        grad_s = (time.time() - t0) / args.steps
        print("adjoint: %.1f ms/step, source gradient: %.1f ms/step" % (1e3 * adj_s, 1e3 * grad_s),
              file=sys.stderr, flush=True)

    default_cfg = (args.n, args.p, args.p_free, args.rhs) == (1000000, 12, 20, 1)
    traffic = (K_M2L_TRAFFIC["fetch_bytes"] + K_M2L_TRAFFIC["write_bytes"]
               if default_cfg and m2l_source_digest() == K_M2L_TRAFFIC["digest"]
               and abs(launches_per_step - K_M2L_TRAFFIC["launches_per_step"]) < 0.5
               and st["m2l_cmac_useful"] == K_M2L_TRAFFIC["m2l_cmac_useful"] else None)

    acc = None
    err_layers = None
    if not args.no_accuracy:
        fn = os.path.join(ROOT, "tests", "golden", "three_%d_sparse400_oracle.npz" % args.n)
        if os.path.exists(fn) and args.rhs == 1:
            g = np.load(fn)
            Js, keep = inputs.sparse_currents(J, 400, seed=0)
            As = fmm.evaluate(torch.tensor(Js, device=dev)).cpu().numpy()
            acc = float(np.linalg.norm(As[g["idx"]] - g["A"]) / np.linalg.norm(g["A"]))
            # per layer (the paper's Err_2 and Err_max over the sampled targets)
            zt = x[g["idx"], 2]
            lay = np.zeros(zt.size, dtype=int)
            for dl in d:
                lay += zt < dl
            err_layers = {}
            for l in range(len(d) + 1):
                sel = lay == l
                if not np.any(sel):
                    continue
                dA, A0 = As[g["idx"]][sel] - g["A"][sel], g["A"][sel]
                err_layers[str(l)] = {
                    "n_sampled": int(sel.sum()),
                    "err2": float(np.linalg.norm(dA) / np.linalg.norm(A0)),
                    "errmax": float(np.max(np.linalg.norm(dA, axis=1) / np.linalg.norm(A0, axis=1)))}
    selfconv = None
    if not args.no_accuracy and not args.no_selfconv and args.rhs == 1:
        # the benchmark's dense currents at every target: the reaction
        # truncation from the evaluation with the reaction order raised
        # (12 -> 16, free part unchanged), the free part's from the free
        # order lowered by two against the benchmark's (an upper bound of
        # its error at the benchmark's order: the error decays geometrically
        # with the order)
        A12 = A[0]
        f16 = lmfmm.LayeredDyadicFMM(d, k, p=args.p + 4, p_free=args.p_free, device=0).build(x)
        A16 = f16.evaluate(Jt.reshape(args.n, 3))
        f16.close()
        f18 = lmfmm.LayeredDyadicFMM(d, k, p=args.p + 4, p_free=args.p_free - 2, device=0).build(x)
        A18 = f18.evaluate(Jt.reshape(args.n, 3))
        f18.close()
        diff = torch.linalg.vector_norm(A12 - A16, dim=1)
        ref = torch.linalg.vector_norm(A16, dim=1)
        dfree = torch.linalg.vector_norm(A18 - A16, dim=1)
        selfconv = {"reaction_orders": [args.p, args.p + 4], "free_orders": [args.p_free - 2, args.p_free],
                    "rel_l2_all_targets": float(torch.linalg.vector_norm(diff).item()
                                                / torch.linalg.vector_norm(ref).item()),
                    "free_part_bound_rel_l2": float(torch.linalg.vector_norm(dfree).item()
                                                    / torch.linalg.vector_norm(ref).item()),
                    "per_layer": {}}
        del A18, dfree
        zt = torch.tensor(x[:, 2], device=dev)
        lay = torch.zeros_like(zt, dtype=torch.int64)
        for dl in d:
            lay += (zt < dl).to(torch.int64)
        for l in range(len(d) + 1):
            sel = lay == l
            selfconv["per_layer"][str(l)] = {
                "err2": float(torch.linalg.vector_norm(diff[sel]).item() / torch.linalg.vector_norm(ref[sel]).item()),
                "errmax": float(torch.max(diff[sel] / ref[sel]).item())}
        del A16, diff, ref
        print("self-convergence (dense currents, all targets): reaction p %d vs %d: %.2e; free part %d vs %d: %.2e" % (
            args.p, args.p + 4, selfconv["rel_l2_all_targets"], args.p_free - 2, args.p_free,
            selfconv["free_part_bound_rel_l2"]), file=sys.stderr, flush=True)
    magnetic = None
    if not args.no_magnetic:
        # magnetic field of the same currents (curl of the electric field); the
        # first call builds the plan without direct reaction pairs
        Jm = torch.tensor(J, device=dev)
        t0 = time.time()
        Hm = fmm.evaluate_h(Jm)
        torch.cuda.synchronize()
        first_s = time.time() - t0
        t0 = time.time()
        for _ in range(args.steps):
            fmm.evaluate_h(Jm, out=Hm)
        torch.cuda.synchronize()
        mag_s = (time.time() - t0) / args.steps
        del Hm, Jm
        magnetic = {"targets_per_s": args.n * args.rhs / mag_s, "ms_per_step": 1e3 * mag_s,
                    "first_call_s": first_s, "vs_forward": (wall / args.steps) / mag_s}
        print("magnetic field: %.1f ms/step (first call %.2f s)" % (1e3 * mag_s, first_s), file=sys.stderr,
              flush=True)
    fmm.close()
    uneven = None if args.no_uneven else uneven_geometries(args, torch, inputs, lmfmm)
    batched = None if args.no_batched else batched_rhs(args, torch, inputs, lmfmm)
    solve = None if args.no_solve else coupled_dipole_solve(args, torch, inputs, lmfmm)
    largest = None if args.no_largest else largest_config(args, torch, inputs, lmfmm)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(d, k, x, J if args.rhs == 1 else J[0], args.n)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "targets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "three-layer dyadic FMM, N=%d uniform in layer slabs, targets=sources, "
                               "p=%d (free-space part p=%d), %d complex128 current vector(s)" % (args.n, args.p, args.p_free or args.p, args.rhs),
                   "n": args.n, "p": args.p, "p_free": args.p_free or args.p, "layers": 3, "n_rhs": args.rhs},
        "roofline": {"bound": "mfma", "kernel": "k_m2l", "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS, "traffic": traffic,
                     "launch_ms": launch_ms, "launches_per_step": launches_per_step,
                     "algorithmic_flops_per_launch": flops_per_launch,
                     "dense_form_flops_per_launch": dense_per_launch,
                     "achieved_dense_equivalent": dense_per_launch / (launch_ms * 1e-3) / 1e12,
                     "executed_flops_per_launch": exec_per_launch,
                     "achieved_executed": achieved_exec,
                     "frac_executed": achieved_exec / FP64_VALU_PEAK_TFLOPS},
        "roofline_kernels": kernels,
        "roofline_path": path,
        "cpu_baseline": cpu,
        "rel_err_vs_oracle": acc,
        "rel_err_vs_oracle_per_layer": err_layers,
        "self_convergence_dense": selfconv,
        "build_s": build_s,
        "cold_targets_per_s": args.n * args.rhs / (build_s + wall / args.steps),
        "trees": trees_roofline(st),
        "phase_ms_per_step": {a: b / max(1, ncalls) for a, b in phases.items()},
        "adjoint": None if adj_s is None else {
            "targets_per_s": args.n * args.rhs / adj_s, "ms_per_step": 1e3 * adj_s,
            "vs_forward": (wall / args.steps) / adj_s},
        "grad_src_xyz": None if grad_s is None else {
            "targets_per_s": args.n * args.rhs / grad_s, "ms_per_step": 1e3 * grad_s,
            "vs_forward": (wall / args.steps) / grad_s},
        "uneven_geometries": uneven,
        "batched_rhs": batched,
        "solve": solve,
        "largest": largest,
        "magnetic": magnetic,
        "m2l_autotune": {"chosen_variant_per_launch": m2l_var,
                         "tuning_ms_per_step_by_variant": [round(float(v), 3) for v in m2l_ms.sum(axis=0)],
                         "tuning_ms_per_step_chosen": round(float(sum(m2l_ms[i, v] for i, v in enumerate(m2l_var))), 3)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
