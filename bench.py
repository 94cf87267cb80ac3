#!/usr/bin/env python3
"""Throughput of sketched Tucker-ALS (Alg. 4) on one MI355X.

Workload (default, zipf10k): sparse 3-way 10000^3 tensor with 1e7 distinct
coordinates drawn per mode from Zipf(1.1), lognormal(0,1) values, FP32; Tucker
rank (16,16,16), TensorSketch with m = 8 * 16^2 = 2048, range-finder
initialisation, 5 sweeps, FP32 operands (FP64 factorisations).  Other
workloads: sparse2000 (2000^3, 1e6 uniform coordinates, rank 10, m = 1600, 10
sweeps) and its leverage-sampling / deterministic-selection variants.  Inputs
are synthetic and seeded (seed 0) and resident in HBM before timing.

One step = one complete call: TensorSketch maps, the sketch pass of every mode
(preparation), range-finder init of modes 2..N, the sweeps of the N sketched
rank-constrained subproblems, and the relative residual after the last sweep.
value = completed sweeps per second of the whole job (sweeps * steps / time).
The phases (preparation, initialisation, sweep loop, residual) are timed
separately with HIP events on the library's stream and reported beside it,
with the sweep loop's own rate.

Prints one JSON line (keys per the benchmark contract) with
  roofline              the launch group that takes the most time, timed live
                        with HIP events on the library's stream over the timed
                        region, against its bound (HBM, matrix cores or vector
                        ALU) with its algorithmic bytes or flops;
  sketch_pass_roofline  the same for the nnz sketch pass (HBM-bound);
  cpu_baseline          the FP64 oracle timed on a bounded sample of the same
                        workload on the host cores.
HBM traffic per launch comes from rocprofv3 FETCH_SIZE / WRITE_SIZE summaries
committed under profiles/ and is reported only while the kernel source they
were taken from is unchanged (else null).
"""
import argparse
import ctypes
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "f64": 78.6}  # dense matrix-core peaks
FP64_VECTOR_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz

# source files whose kernels make up each launch group (for the traffic check)
GROUP_SOURCES = {
    "sketch_pass": ["sketch_pass.hip"], "rrf_pass": ["sketch_pass.hip", "rrf_dense.hip"],
    "ts_lhs": ["ts_lhs.hip"], "gram": ["gemm.hip"], "solve_la": ["linalg.hip", "gemm.hip"],
    "eig": ["linalg.hip"], "fit": ["fit.hip"], "rrf": ["linalg.hip", "gemm.hip", "api.hip"],
    "leverage": ["leverage.hip"], "fiber_index": ["fibers.hip"], "fiber_rows": ["fibers.hip"],
    "select": ["select.hip"], "cp_core": ["cp.hip", "fit.hip"],
}
GROUPS = ["sketch_pass", "rrf_pass", "rrf", "ts_lhs", "gram", "solve_la", "eig", "fit",
          "leverage", "fiber_index", "fiber_rows", "select", "cp_core"]
WORKLOADS = ["zipf10k", "sparse2000", "sparse2000lev", "sparse2000det", "dense4d200", "cp500",
             "dense40"]
PHASES = ["phase_prep", "phase_init", "phase_sweeps", "phase_fit"]


# The test tensors of Sec. 7 with the experiments' parameters: name -> (builder
# of (dense | (idx, val)), s, R, description).
PAPER_TENSORS = {
    "t1a12": ("dense", 200, 5, "Tensor 1, s=200, R=5, alpha=1.2"),
    "t1a16": ("dense", 200, 5, "Tensor 1, s=200, R=5, alpha=1.6"),
    "t2": ("dense", 200, 5, "Tensor 2 (power-law spikes), s=200, R=5, alpha=1.6"),
    "t3": ("sparse", 2000, 10, "Tensor 3, s=2000, R=10, alpha=1.2, p=0.02"),
    "t4": ("dense", 200, 5, "Tensor 4 on Tensor 1 (10 coherent entries), s=200, R=5, alpha=1.6"),
    "t4s": ("sparse", 2000, 10, "Tensor 4 on Tensor 3, s=2000, R=10, alpha=1.2, p=0.02"),
}


def paper_tensor(name, seed):
    import workloads as W
    return {"t1a12": lambda: W.paper_tensor1(200, 5, 1.2, seed),
            "t1a16": lambda: W.paper_tensor1(200, 5, 1.6, seed),
            "t2": lambda: W.paper_tensor2(200, 5, 1.6, seed),
            "t3": lambda: W.paper_tensor3(2000, 10, 1.2, 0.02, seed),
            "t4": lambda: W.paper_tensor4_dense(200, 5, 1.6, seed),
            "t4s": lambda: W.paper_tensor4_sparse(2000, 10, 1.2, 0.02, seed)}[name]()


def fitness_vs_k(args):
    """Final fitness 1 - ||T - T~|| / ||T|| after 5 sweeps (the experiments'
    count) for TensorSketch, leverage sampling and deterministic leverage
    selection, RRF and random initialisation, m = K R^2, FP64 operands, on
    `seeds` tensors of the chosen family (tensor seed = run seed).  Dense
    tensors also get the unsketched ALS from the RRF start (every row kept)."""
    import statistics
    import torch
    import paper_2104_01101_amd as tsk
    from paper_2104_01101_amd import _lib as L
    dev = torch.device("cuda:0")
    layout, s, R, desc = PAPER_TENSORS[args.fitness]
    ks = [int(k) for k in args.ks.split(",")]
    res = {}
    t0 = time.perf_counter()
    for seed in range(args.seeds):
        data = paper_tensor(args.fitness, seed)
        if layout == "dense":
            T = tsk.Tensor.dense(torch.from_numpy(data).to(dev))
        else:
            idx, val = data
            T = tsk.Tensor.coo(torch.from_numpy(idx).to(dev), torch.from_numpy(val).to(dev),
                               (s, s, s))
        runs = [(kind, init, K) for K in ks for kind in ("ts", "lev", "lev_det")
                for init in ("rrf", "random")]
        if layout == "dense":
            runs.append(("lev_det", "rrf", s * s // (R * R)))  # every row: unsketched ALS
        for kind, init, K in runs:
            try:
                _, _, fits = tsk.tucker_sketch_als(T, (R, R, R), K * R * R, 5, sketch=kind,
                                                   init=init, prec="f64", seed=seed,
                                                   solve=args.solve)
                f = 1.0 - fits[-1]
            except L.TskError as e:  # singular sketched Gram: the sketch missed the signal
                if e.status != L.ENUMERIC:
                    raise
                f = None
            res.setdefault((kind, init, K), []).append(f)
        del T
        torch.cuda.empty_cache()
    for (kind, init, K), fs in res.items():
        f = [v for v in fs if v is not None]
        print(json.dumps({"tensor": args.fitness, "description": desc, "method": kind,
                          "init": init, "K": K, "m": K * R * R, "sweeps": 5,
                          "solve": args.solve, "seeds": len(fs),
                          "breakdowns": len(fs) - len(f),
                          "fitness_mean": statistics.fmean(f) if f else None,
                          "fitness_min": min(f) if f else None,
                          "fitness_max": max(f) if f else None,
                          "unsketched": K * R * R == s * s}))
    print(json.dumps({"tensor": args.fitness, "runs": sum(len(v) for v in res.values()),
                      "seconds": time.perf_counter() - t0}))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="zipf10k", choices=WORKLOADS,
                    help="zipf10k (default: 10000^3, 1e7 Zipf entries, rank 16, m = 2048), "
                         "sparse2000 (2000^3, 1e6 uniform entries, rank 10, m = 1600), "
                         "sparse2000lev / sparse2000det (the same tensor under "
                         "leverage-score sampling / deterministic leverage selection, "
                         "through the fibre indices), dense4d200 (dense 200^4, rank 10, "
                         "leverage m = 4000), cp500 (dense 500^3 CP rank 20, leverage "
                         "Tucker to rank 30, m = 14400, then CP-ALS on the core)")
    ap.add_argument("--solve", default="rsvd", choices=["rsvd", "exact"],
                    help="subproblem solver: rsvd = RSVD-LRLS (Alg. 5, the solver Alg. 4 "
                         "calls) or exact = truncated SVD of Z^+ Y")
    ap.add_argument("--prec", default=None, choices=["f32", "bf16", "f64"],
                    help="operand precision of the sketched products (default: the workload's, "
                         "FP32); bf16 = BF16 operands with FP32 accumulation")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--breakdown", action="store_true",
                    help="also print per-group times of the last warm-up step (stderr)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy kernel (counter scale)")
    ap.add_argument("--fitness", default=None, choices=sorted(PAPER_TENSORS),
                    help="instead of the benchmark: final fitness against the sketch size "
                         "parameter K on one of the paper's test tensors (one JSON line per "
                         "method, initialisation and K)")
    ap.add_argument("--ks", default="4,8,16", help="K values of --fitness (m = K R^2)")
    ap.add_argument("--seeds", type=int, default=3, help="random seeds per point of --fitness")
    return ap.parse_args()


def workload(name):
    import workloads
    return getattr(workloads, name)()


def group_work(w, solve="exact"):
    """Algorithmic work of one job per launch group: name -> (bound, amount, peak, unit).
    bytes for HBM-bound groups, flops otherwise."""
    import numpy as np
    N = len(w.dims)
    s, R, m, sweeps = w.dims[0], w.ranks[0], w.m, w.sweeps
    dense = w.dense is not None
    nnz = w.dense.size if dense else w.val.shape[0]
    ib = 0 if dense else 4 * N  # index bytes per stored entry
    r = R ** (N - 1)
    q = min(r, s)
    k1 = math.ceil(math.sqrt(m / r) * R - 1e-9)
    k2 = R * R + k1
    # tensor values (and the sketched right-hand sides of the pass): FP32, or FP64
    vb = 8 if (w.dense if dense else w.val).dtype == np.float64 else 4
    vo = {"f32": 4, "bf16": 2, "f64": 8}[w.prec]  # operand bytes of Z and sampled Y
    subs = N * sweeps
    pk = PEAK_TFLOPS[w.prec]
    eig = lambda n: 4.0 / 3.0 * n ** 3 + 2.0 * n * n * R
    kk = min(R + 10, r)  # RSVD-LRLS test-matrix columns
    # the library's choice of product order (solve.hip): the fused chain for
    # r <= 128, k <= 24; otherwise the O(m s k) order when r >= 4k
    yside = solve == "rsvd" and not (r <= 128 and kk <= 24) and r >= 4 * kk
    gram = 2.0 * m * r * (r + s)  # [Z^T Z; Y^T Z]
    if yside:
        gram = 2.0 * m * r * r + 4.0 * m * s * kk  # Z^T Z, Y Omega, Y^T (Z P)
        # inverse, C0 = Z^T (Y Omega), C^T = C0^T B, thin QR, B Q, Z P, D D^T (FP64)
        la = r ** 3 + 2.0 * m * r * kk + 4.0 * kk * r * r + 4.0 * kk * kk * r \
            + 2.0 * m * r * kk + 2.0 * kk * kk * s
        q_eig = kk
    elif solve == "rsvd":
        # inverse, Om^T H^T, C^T, thin QR, B Q, D^T, D D^T (FP64)
        la = r ** 3 + 2.0 * kk * r * s + 4.0 * kk * r * r + 4.0 * kk * kk * r \
            + 2.0 * s * r * kk + 2.0 * kk * kk * s
        q_eig = kk
    else:
        # Gram inverse, X = H G^-1, X X^T, A = X^T U, W = X A (FP64)
        la = r ** 3 + 4.0 * s * r * q + 4.0 * s * r * R
        q_eig = q
    return {
        # COO stream (N int32 indices + value) read once, every Y^(n) written once
        "sketch_pass": ("hbm", nnz * (ib + vb) + N * m * s * vb, HBM_PEAK_GBS, "GB/s"),
        # sparse: one pass over the entries writing W; dense: the tensor read
        # once per initialised mode by the structured GEMM
        "rrf_pass": (("hbm", (N - 1) * nnz * vb, HBM_PEAK_GBS, "GB/s") if dense else
                     ("hbm", nnz * (ib + vb) + (N - 1) * k2 * s * vb, HBM_PEAK_GBS, "GB/s")),
        # B = W G (s x k2 x k1) and the Gram of B, per initialised mode
        "rrf": ("mfma", (N - 1) * (2.0 * s * k2 * k1 + 2.0 * s * k1 * k1),
                PEAK_TFLOPS["f64"], "TFLOP/s"),
        # CountSketches read, Z written
        "ts_lhs": ("hbm", subs * ((N - 1) * s * R * 8 + m * r * vo), HBM_PEAK_GBS, "GB/s"),
        # G = Z^T Z and Z^T Y (or the two products with Y in the O(m s k) order)
        "gram": ("mfma", subs * gram, pk, "TFLOP/s"),
        "solve_la": ("mfma", subs * la, PEAK_TFLOPS["f64"], "TFLOP/s"),
        # tridiagonalisation + back-transformation of R vectors (FP64 vector ALU)
        "eig": ("alu", subs * eig(q_eig) + (N - 1) * eig(k1), FP64_VECTOR_TFLOPS, "TFLOP/s"),
        # after the last sweep: dense, the tensor read once; sparse order 3 of
        # rank 16 from 2^16 entries (entries grouped by their last index),
        # W = C x_3 A^(3) and R^2 multiply-adds per entry on the FP64 matrix
        # cores; other sparse shapes, per entry the core contraction
        # R^3 + R^2 + R multiply-adds (FP64 vector ALU)
        "fit": (("hbm", nnz * vb, HBM_PEAK_GBS, "GB/s") if dense else
                ("mfma", 2.0 * (nnz * R ** 2 + s * R ** 3), PEAK_TFLOPS["f64"], "TFLOP/s")
                if N == 3 and R == 16 and all(x == R for x in w.ranks) and nnz >= (1 << 16) else
                ("alu", nnz * 2.0 * (R ** 3 + R ** 2 + R), FP64_VECTOR_TFLOPS, "TFLOP/s")),
        # CP-ALS on the core and the CP residual against the dense tensor
        "cp_core": ("hbm", nnz * vb, HBM_PEAK_GBS, "GB/s"),
        # sampled Kronecker rows: factors read, Z written
        "leverage": ("hbm", subs * ((N - 1) * s * R * 8 + m * r * vo), HBM_PEAK_GBS, "GB/s"),
        # per mode: keys built (indices read, keys written), then sorted pairs written once
        "fiber_index": ("hbm", N * nnz * (4 * N + 8 + 12), HBM_PEAK_GBS, "GB/s"),
        # deterministic selection: candidate products and their sort keys (about
        # m (ln m + 1) candidates, 8-byte key + 4-byte id written, sorted, read back)
        "select": ("hbm", subs * 3 * m * (math.log(m) + 1) * 24, HBM_PEAK_GBS, "GB/s"),
        # sampled fibres: Y written, the fibres' keys and values read (expected length
        # nnz / prod_{k != n} s_k), sample indices and weights read
        "fiber_rows": ("hbm", subs * (m * s * vo + m * (nnz / s ** (N - 1)) * 12
                                      + m * (4 * (N - 1) + 8)), HBM_PEAK_GBS, "GB/s"),
    }


def source_digest(group):
    h = hashlib.sha256()
    for f in GROUP_SOURCES.get(group, []):
        with open(os.path.join(ROOT, "paper_2104_01101_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic(group, wname):
    """HBM bytes per launch from a committed counter summary, if still current."""
    path = os.path.join(ROOT, "profiles", f"traffic_{group}_{wname}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256_16") != source_digest(group):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline(name, work, ms_total, launches, steps, wname):
    bound, amount, peak, unit = work[name]
    secs = ms_total / 1e3
    per_launch = amount * steps / max(1, launches)
    if unit == "GB/s":
        achieved = amount * steps / secs / 1e9
    else:
        achieved = amount * steps / secs / 1e12
    t = traffic(name, wname)
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": t, "kernel": name,
            "algorithmic_per_launch": per_launch, "avg_launch_ms": ms_total / max(1, launches),
            "launches": launches}


def adjoint_timing(tsk, L, lib, read, w, reps=5):
    """Sketched mode-0 residual (forward) and its adjoint (backward) at the
    shape of this job's subproblem (m x s_0 FP32 Y, r = prod of the other
    ranks, R = R_0), seeded inputs.  Whole calls are timed with events on the
    launching stream; the pass over Y (one launch per call) with the library's
    own events.  Backward pass: 6 m s R FP64 flops on the matrix cores
    (E = P A^T - Y, E^T P, E A); forward: Y read once (HBM)."""
    import numpy as np
    import torch
    dims, ranks, m, n = tuple(w.dims), tuple(w.ranks), w.m, 0
    s, R = dims[n], ranks[n]
    g = torch.Generator(device="cuda:0").manual_seed(5)
    fg = [torch.randn((d, r), dtype=torch.float64, device="cuda:0", generator=g) / d ** 0.5
          for d, r in zip(dims, ranks)]
    cg = torch.randn(ranks, dtype=torch.float64, device="cuda:0", generator=g)
    Y = torch.randn((m, s), dtype=torch.float32, device="cuda:0", generator=g)
    h, sg = tsk.hash_tables(dims, n, m, 3)
    res = {}
    for name, call in (("fwd", lambda: tsk.sketched_residual(dims, ranks, n, m, h, sg, fg, cg, Y)),
                       ("bwd", lambda: tsk.sketched_residual_grads(dims, ranks, n, m, h, sg, fg,
                                                                   cg, Y))):
        call()
        torch.cuda.synchronize()
        L.check(lib.tsk_profile_enable(b"adjoint_pass"))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms, launches = read("adjoint_pass")
        L.check(lib.tsk_profile_enable(b""))
        if launches == 0:
            raise RuntimeError("no timed launches of the adjoint pass were recorded")
        per = ms / launches
        if name == "fwd":
            amount, bound, peak, unit = m * s * 4 + (m + s) * R * 8, "hbm", 8000.0, "GB/s"
            achieved = amount / (per / 1e3) / 1e9
        else:
            amount, bound, peak, unit = 6 * m * s * R, "mfma", 78.6, "TFLOP/s"
            achieved = amount / (per / 1e3) / 1e12
        res[name] = {"call_ms": e0.elapsed_time(e1) / reps,
                     "pass": {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                              "frac": achieved / peak, "algorithmic_per_launch": amount,
                              "avg_launch_ms": per, "launches": launches}}
    res["shape"] = f"m={m}, s={s}, r={int(np.prod(ranks[1:]))}, R={R}, FP32 Y, FP64 arithmetic"
    return res


def copy_calibration():
    import torch
    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.fitness:
        fitness_vs_k(args)
        return
    import torch
    import paper_2104_01101_amd as tsk
    from paper_2104_01101_amd import _lib as L

    dev = torch.device("cuda:0")
    w = workload(args.workload)
    if args.prec:
        w["prec"] = args.prec
    dense = w.dense is not None
    if dense:
        T = tsk.Tensor.dense(torch.from_numpy(w.dense).to(dev))
    else:
        T = tsk.Tensor.coo(torch.from_numpy(w.idx).to(dev), torch.from_numpy(w.val).to(dev),
                           w.dims)
    cp = w.get("cp_rank") is not None
    if cp:  # Alg. 6: the job is CP-Sketch-Tucker; its CP residual is the result
        class _CpJob:
            def run(self):
                _, f = tsk.cp_via_tucker(T, w.cp_rank, w.ranks, w.m, w.sweeps, w.cp_sweeps,
                                         sketch=w.sketch, prec=w.prec, seed=0, solve=args.solve)
                return None, None, [f]
        plan = _CpJob()
    else:
        plan = tsk.TuckerPlan(T, w.ranks, w.m, w.sweeps, sketch=w.sketch, init="rrf",
                              prec=w.prec, seed=0, record_fit="final", solve=args.solve)
    second = ("sketch_pass" if w.sketch == "ts" else "rrf_pass" if dense else "fiber_rows")
    lib = L.lib()
    lib.tsk_profile_enable.argtypes = [ctypes.c_char_p]
    lib.tsk_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64)]

    def read(name):
        ms, n = ctypes.c_double(0), ctypes.c_int64(0)
        L.check(lib.tsk_profile_read(name.encode() if name else None, ctypes.byref(ms),
                                     ctypes.byref(n)))
        return ms.value, n.value

    # warm-up; the last warm-up step is profiled per group to find the dominant one
    nw = max(1, args.warmup)
    for i in range(nw):
        if i == nw - 1:
            L.check(lib.tsk_profile_enable(b"*"))
        plan.run()
    per_group = {n: read(n) for n in GROUPS}
    L.check(lib.tsk_profile_enable(b""))
    dominant = max(per_group, key=lambda n: per_group[n][0])
    if args.breakdown:
        print(json.dumps({"breakdown_ms_per_step": {n: round(v[0], 4) for n, v in per_group.items()},
                          "launch_groups": {n: v[1] for n, v in per_group.items()}}),
              file=sys.stderr)

    # timed region: the dominant group's and the sketch pass's (leverage:
    # the fibre gather's) launches are timed with events on the library's stream
    timed = ",".join(dict.fromkeys([dominant, second] + PHASES))
    L.check(lib.tsk_profile_enable(timed.encode()))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fits = None
    for _ in range(args.steps):
        _, _, fits = plan.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dom = read(dominant)
    sp = read(second)
    phases = {p: read(p)[0] / args.steps for p in PHASES}
    L.check(lib.tsk_profile_enable(b""))

    work = group_work(w, args.solve)
    out = {
        "metric": "ALS sweeps/s + sketch-pass GB/s at fixed relative residual, FP32 vs BF16/adjoint",
        "value": w.sweeps * args.steps / elapsed,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.prec,
        "data": "synthetic",
        "config": {"workload": {
                       "sparse2000": "sparse 2000^3, 1e6 nnz uniform, Tucker rank 10 + N(0,1), "
                                     "TensorSketch m=1600, RRF init, 10 sweeps of Alg. 4, "
                                     "FP32 operands",
                       "sparse2000lev": "sparse 2000^3, 1e6 nnz uniform, Tucker rank 10 + "
                                        "N(0,1), leverage-score sampling m=1600 through "
                                        "per-mode fibre indices, RRF init, 10 sweeps of "
                                        "Alg. 4, FP32 operands",
                       "sparse2000det": "sparse 2000^3, 1e6 nnz uniform, Tucker rank 10 + "
                                        "N(0,1), deterministic leverage selection m=2400 "
                                        "through per-mode fibre indices, RRF init, 10 sweeps "
                                        "of Alg. 4, FP32 operands",
                       "zipf10k": "sparse 10000^3, 1e7 nnz Zipf(1.1), lognormal values, "
                                  "Tucker rank 16, TensorSketch m=2048, RRF init, 5 sweeps, "
                                  "FP32 operands",
                       "dense4d200": "dense 200^4 FP32 (6.4 GB), Tucker rank 10 + 1% noise, "
                                     "leverage-score sampling m=4000, RRF init, 5 sweeps of "
                                     "Alg. 4, FP32 operands",
                       "dense40": "dense 40^3 FP64, Tucker rank 5 + 1% noise, TensorSketch "
                                  "m=200, RRF init, 5 sweeps of Alg. 4, FP64 operands",
                       "cp500": "dense 500^3 FP32, CP rank 20 (collinearity 0.9) + 1% noise; "
                                "Alg. 6: leverage-sampled Tucker to rank 30 (m=14400, RRF "
                                "init, 5 sweeps), CP-ALS rank 20 on the core (25 sweeps), "
                                "FP32 operands"}[args.workload].replace(
                       "FP32 operands", {"f32": "FP32", "bf16": "BF16 (FP32-accumulated)",
                                         "f64": "FP64"}[w.prec] + " operands"),
                   "dims": list(w.dims),
                   "nnz": int(w.dense.size if dense else w.val.shape[0]), "ranks": list(w.ranks),
                   "m": w.m, "sweeps": w.sweeps, "prec": w.prec,
                   "solve": "RSVD-LRLS (Alg. 5)" if args.solve == "rsvd" else "exact truncated SVD"},
        ("final_cp_relative_residual" if cp else "final_relative_residual"):
            fits[-1] if fits else None,
        "phases_ms_per_step": {p[6:]: round(v, 4) for p, v in phases.items()},
        "sweep_loop_sweeps_per_s": (w.sweeps / (phases["phase_sweeps"] / 1e3)
                                    if phases["phase_sweeps"] > 0 else None),
        "roofline": roofline(dominant, work, dom[0], dom[1], args.steps, args.workload),
        f"{second}_roofline": roofline(second, work, sp[0], sp[1], args.steps, args.workload),
    }
    if args.workload == "zipf10k":
        out["adjoint"] = adjoint_timing(tsk, L, lib, read, w, reps=max(3, args.steps))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = (cpu_baseline_whole(w, args.solve) if args.workload == "dense40"
                               else cpu_baseline_dense(w, args.solve) if dense else
                               cpu_baseline(w, args.solve, 1 if args.workload == "zipf10k" else 3))
    print(json.dumps(out))


def cpu_baseline(w, solve="exact", sample_sweeps=3):
    """FP64 oracle on the same input: preparation (maps, sketched right-hand
    sides, range finder), `sample_sweeps` of the sweeps and one relative
    residual are timed; the job time is extrapolated to preparation + all
    sweeps + the residual after the last one (what the GPU job computes)."""
    import numpy as np
    from oracle import sketch as osk, solve as osv, tucker as otk
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    T = osk.Tensor(w.dims, w.idx, w.val.astype(np.float64))
    N, m, ranks, seed = len(w.dims), w.m, w.ranks, 0
    ts = w.sketch == "ts"
    t0 = time.perf_counter()
    if ts:
        tables = {n: osk.ts_tables(w.dims, m, seed, n) for n in range(N)}
        Ys = {n: osk.ts_rhs(T, m, tables[n], n) for n in range(N)}
    factors = [None] * N
    for n in range(1, N):
        k1, k2 = otk.default_rrf_sizes(m, ranks, n)
        factors[n] = otk.init_rrf(T, n, ranks[n], k1, k2, seed)
    t_prep = time.perf_counter() - t0
    t1 = time.perf_counter()
    for sweep in range(sample_sweeps):
        for n in range(N):
            if ts:
                Z, Y = osk.ts_lhs(factors, tables[n], m, n), Ys[n]
            else:
                idx, wt = (osk.leverage_select(factors, m, n) if w.sketch == "lev_det"
                           else osk.leverage_sample(factors, m, seed, sweep, n))
                Z = osk.leverage_lhs(factors, idx, wt, n)
                Y = osk.leverage_rhs_sparse(T, idx, wt, n)
            if solve == "rsvd":
                kk = otk.rsvd_width(ranks[n], Z.shape[1])
                Om = otk.rsvd_omega(seed, sweep, n, w.dims[n], kk)
                A, W = osv.rsvd_lrls(Z, Y, ranks[n], Om)
            else:
                A, W, _ = osv.rc_solve(Z, Y, ranks[n])
            factors[n] = A
            core = otk.W_to_core(W, ranks, n)
    t_sweep = (time.perf_counter() - t1) / sample_sweeps
    t2 = time.perf_counter()
    otk.relative_residual(T, core, factors)
    t_fit = time.perf_counter() - t2
    job = t_prep + w.sweeps * t_sweep + t_fit
    return {"value": w.sweeps / job, "unit": "sweeps/s", "cores": int(cores), "kind": "oracle",
            "sample": f"full input; preparation ({t_prep:.2f} s), {sample_sweeps} of "
                      f"{w.sweeps} sweeps ({t_sweep:.2f} s each) and one residual "
                      f"({t_fit:.2f} s) timed, job = preparation + {w.sweeps} sweeps + "
                      f"residual"}


def cpu_baseline_whole(w, solve="rsvd"):
    """FP64 oracle running the whole job (small workloads): maps, sketched
    right-hand sides, range finder, every sweep and the final residual."""
    import numpy as np
    from oracle import sketch as osk, tucker as otk
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    T = osk.Tensor.from_dense(np.asarray(w.dense, dtype=np.float64))
    t0 = time.perf_counter()
    ref = otk.sketch_tucker_als(T, w.ranks, w.m, w.sweeps, seed=0, sketch_kind=w.sketch,
                                solve_kind=solve, record_fit=False)
    secs = time.perf_counter() - t0
    res = otk.relative_residual(T, ref["core"], ref["factors"])
    return {"value": w.sweeps / secs, "unit": "sweeps/s", "cores": cores, "kind": "oracle",
            "sample": f"the whole job ({w.sweeps} sweeps, final residual {res:.10f})"}


def cpu_baseline_dense(w, solve="rsvd", slab=0.02):
    """FP64 oracle on a bounded sample of a dense workload: one sweep of the
    leverage-sampled subproblems on the full tensor (from random orthonormal
    factors), and the range finder of one mode and the residual on a slab of
    the first `slab` of the mode-0 slices, scaled by the entry count to all
    the range-finder modes and the whole tensor."""
    import numpy as np
    from oracle import sketch as osk, solve as osv, tucker as otk
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    X, N, m, ranks = w.dense, len(w.dims), w.m, w.ranks
    rs = np.random.default_rng(0)
    factors = [np.linalg.qr(rs.standard_normal((d, R)))[0] for d, R in zip(w.dims, ranks)]
    t0 = time.perf_counter()
    for n in range(N):
        idx, wt = osk.leverage_sample(factors, m, 0, 0, n)
        Z = osk.leverage_lhs(factors, idx, wt, n)
        Y = osk.leverage_rhs_dense(X, idx, wt, n)
        if solve == "rsvd":
            kk = otk.rsvd_width(ranks[n], Z.shape[1])
            A, W = osv.rsvd_lrls(Z, Y, ranks[n], otk.rsvd_omega(0, 0, n, w.dims[n], kk))
        else:
            A, W, _ = osv.rc_solve(Z, Y, ranks[n])
        factors[n] = A
        core = otk.W_to_core(W, ranks, n)
    t_sweep = time.perf_counter() - t0
    rows = max(1, int(round(slab * w.dims[0])))
    Xs = np.ascontiguousarray(X[:rows], dtype=np.float64)
    scale = X.shape[0] / rows
    Ts = osk.Tensor.from_dense(Xs)
    t1 = time.perf_counter()
    k1, k2 = otk.default_rrf_sizes(m, ranks, 1)
    otk.init_rrf(Ts, 1, ranks[1], k1, k2, 0)
    t_rrf = (time.perf_counter() - t1) * scale * (N - 1)
    fs = [factors[0][:rows]] + factors[1:]
    t2 = time.perf_counter()
    otk.relative_residual(Ts, core, fs)
    t_fit = (time.perf_counter() - t2) * scale
    job = t_rrf + w.sweeps * t_sweep + t_fit
    return {"value": w.sweeps / job, "unit": "sweeps/s", "cores": int(cores), "kind": "oracle",
            "sample": f"one sweep of the {N} leverage-sampled subproblems on the full tensor "
                      f"({t_sweep:.2f} s); range finder of one mode and the residual on "
                      f"{rows} of {w.dims[0]} mode-0 slices, scaled by entries to "
                      f"{N - 1} modes ({t_rrf:.2f} s) and the whole tensor ({t_fit:.2f} s); "
                      f"job = range finder + {w.sweeps} sweeps + residual"
                      + ("; the CP-ALS on the 30^3 core is not timed" if
                         w.get("cp_rank") else "")}


if __name__ == "__main__":
    main()
