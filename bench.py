"""Benchmark of the NNLS hot path on one MI355X.

One step = the whole path of Algorithm 1 on one resident instance of the large single
right-hand-side workload (A 20000 x 5000 FP32, U[0,1] entries, 70 % zeros in x, 1 % noise):
column scales -> BF16x3 Gram with fused rescale -> Algorithm 2 (whole-GPU solver, Q held in
registers) -> FP64 KKT check and refinement step.  The inputs are generated on the host, copied
to HBM before the timed region, and every step writes into preallocated buffers (no allocation
while timed).

Prints one JSON line: solves/s (value), per-call milliseconds, the roofline of the dominant
kernel measured with HIP events on the library's stream, and the FP64 oracle timed on a bounded
column sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2516.6
PEAK_BF16X3_TFLOPS = PEAK_BF16_TFLOPS / 3.0   # three bf16 products per FP32-equivalent product
TOL = 1e-5
# The solve runs to 0.8 tol in FP32 on the BF16x3 Q; the FP64 check against (A, b) is what
# must meet tol (it differs from the FP32 residual by ~1e-7 at this workload).
INNER_TOL = 8e-6
BATCH_INNER_TOL = 5e-6
BATCH_MAX_ITER = 20000
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
# learned warm start: training recipe (the method's own solves of 200k seeded b = A x)
WARM_TRAIN = 200000
WARM_EVAL = 32768
WARM_TARGET_TOL = 3e-6
WARM_EPOCHS = 60
WARM_BATCH = 512
WARM_LR = 1e-3
WARM_LAMBDA = 1e-4
MLP_FWD_FLOP = 2.0 * (256 * 1024 + 1024 * 1024 + 1024 * 256)   # per sample


CSRC = os.path.join(ROOT, "paper_1502_01645_amd", "csrc")


def _src_sha(src):
    """Hash of a kernel's source file together with every shared header of the library."""
    h = hashlib.sha256()
    headers = sorted(f for f in os.listdir(CSRC) if f.endswith(".hpp"))
    for name in [src] + headers:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record(kernel_key, src):
    """Measured HBM traffic per launch of a kernel (rocprofv3 FETCH_SIZE + WRITE_SIZE, each
    scaled by what the counter reads for a copy kernel of known size) if it was taken on the
    current source of that kernel; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel_key)
    if not rec or rec.get("source_sha") != _src_sha(src):
        return None
    return rec.get("bytes_per_launch")


def stage_rooflines(N, d, n, k, ms, rows_read):
    """Rooflines of the prepare call (BF16x3 Gram flops d n (n + 1) + 2 d n k over the call's
    time) and of the single-RHS solver (4 n bytes per row of Q a streaming solver reads, over the
    solve time); returns (dominant, other) by time."""
    gram_tf = (d * n * (n + 1) + 2.0 * d * n * k) / (ms["prepare"] * 1e-3) / 1e12
    solve_gbs = 4.0 * n * rows_read / (ms["solve"] * 1e-3) / 1e9
    solver = N.solver_name(n, k, N.F32)
    kern = {"regq": "solve_regq_kernel", "persistent": "solve_persistent_kernel"}.get(
        solver, "solve_" + solver + "_kernel")
    rg = {"kernel": "gram_dma_kernel", "timed": "nnls_prepare call", "bound": "mfma",
          "achieved": round(gram_tf, 2), "peak": round(PEAK_BF16X3_TFLOPS, 1),
          "unit": "TFLOP/s", "frac": round(gram_tf / PEAK_BF16X3_TFLOPS, 4), "traffic": None}
    rs = {"kernel": kern, "bound": "hbm", "achieved": round(solve_gbs, 1), "peak": PEAK_HBM_GBS,
          "unit": "GB/s", "frac": round(solve_gbs / PEAK_HBM_GBS, 4), "traffic": None}
    return (rg, rs) if ms["prepare"] >= ms["solve"] else (rs, rg)


def cpu_baseline(A, b, n_full, iters_full, cols):
    """The FP64 oracle on the first `cols` columns of the workload (same b): Gram, rescale and
    Algorithm 2, each timed; a full-size solve is extrapolated with the Gram's d n (n+1) cost and
    the per-iteration n^2 cost times the iterations the GPU solve needed at full size."""
    from oracle import oracle as O
    orc = O.load()
    As = np.ascontiguousarray(A[:, :cols], dtype=np.float64)
    bs = b.astype(np.float64)
    t0 = time.perf_counter()
    H, h = orc.gram(As, bs)
    t_gram = time.perf_counter() - t0
    s, Q, q = orc.rescale(H, h)
    t0 = time.perf_counter()
    y, it, kkt, st = orc.nqp(Q, q[:, 0], TOL, 100000)
    t_solve = time.perf_counter() - t0
    m = cols
    t_iter = t_solve / max(it, 1)
    t_full = (t_gram * (n_full * (n_full + 1)) / (m * (m + 1))
              + t_iter * (n_full / m) ** 2 * iters_full)
    return {
        "value": 1.0 / t_full,
        "unit": "solves/s",
        "cores": orc.num_threads(),
        "kind": "oracle",
        "sample": (f"oracle Gram+rescale+Algorithm 2 on the first {m} of {n_full} columns "
                   f"(d={A.shape[0]}): gram {t_gram:.2f} s, {it} iterations {t_solve:.2f} s; "
                   f"full solve extrapolated as gram*n(n+1)/(m(m+1)) + per-iteration*(n/m)^2*"
                   f"{iters_full} iterations = {t_full:.1f} s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample-cols", type=int, default=1400)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="large",
                    choices=["large", "manyrhs", "batched", "warm", "ablation", "paper", "nmf"])
    ap.add_argument("--epochs", type=int, default=WARM_EPOCHS)
    ap.add_argument("--batch", type=int, default=8192)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.workload == "manyrhs":
        return bench_manyrhs(args)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "warm":
        return bench_warm(args)
    if args.workload == "ablation":
        return bench_ablation(args)
    if args.workload == "paper":
        return bench_paper(args)
    if args.workload == "nmf":
        return bench_nmf(args)

    import torch
    from paper_1502_01645_amd import nnls as N
    from paper_1502_01645_amd import workloads as W

    dev = torch.device("cuda:0")
    A_h, b_h, _ = W.make_large()
    d, n = A_h.shape
    k = 1
    A = torch.from_numpy(A_h).to(dev)
    b = torch.from_numpy(b_h).to(dev)

    # preallocated outputs and workspaces
    s = torch.empty(n, dtype=torch.float64, device=dev)
    Q = torch.empty((n, n), dtype=torch.float32, device=dev)
    q = torch.empty((n, k), dtype=torch.float32, device=dev)
    X = torch.empty((n, k), dtype=torch.float32, device=dev)
    iters = torch.empty(k, dtype=torch.int32, device=dev)
    kkt = torch.empty(k, dtype=torch.float64, device=dev)
    status = torch.empty(k, dtype=torch.int32, device=dev)
    rows = torch.zeros(k, dtype=torch.int64, device=dev)
    steps_total = args.warmup + args.steps
    kkt64 = torch.empty((steps_total, k), dtype=torch.float64, device=dev)
    obj64 = torch.empty((steps_total, k), dtype=torch.float64, device=dev)
    ws_p = torch.empty(max(N.workspace_bytes(N.OP_PREPARE, d, n, k, N.GRAM_BF16X3, N.F32), 1),
                       dtype=torch.uint8, device=dev)
    ws_v = torch.empty(max(N.workspace_bytes(N.OP_SOLVE, d, n, k, 0, N.F32), 1), dtype=torch.uint8,
                       device=dev)
    ws_r = torch.empty(max(N.workspace_bytes(N.OP_REFINE, d, n, k, 0, N.F32), 1), dtype=torch.uint8,
                       device=dev)
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    marks = [[ev() for _ in range(4)] for _ in range(steps_total)]

    def step(i):
        e = marks[i]
        e[0].record()
        N.prepare(A, b, N.GRAM_BF16X3, out=(Q, q, s), ws=ws_p)
        e[1].record()
        N.solve(Q, q, s, tol=INNER_TOL, max_iter=5 * n, out=(X, iters, kkt, status), ws=ws_v,
                rows_read=rows)
        e[2].record()
        N.refine(A, b, X, out=(kkt64[i], obj64[i]), ws=ws_r)
        e[3].record()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, steps_total):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    timed = marks[args.warmup:]
    ms = {name: float(np.mean([m[j].elapsed_time(m[j + 1]) for m in timed]))
          for j, name in enumerate(["prepare", "solve", "refine"])}
    ms_step = wall * 1e3 / args.steps
    r64 = kkt64[args.warmup:].cpu().numpy()[:, 0]
    ok = bool(np.all(r64 <= TOL))
    it_last = int(iters.cpu()[0])
    rows_last = int(rows.cpu()[0])
    st_last = int(status.cpu()[0])

    # roofline of the two heavy kernels
    gram_flops = d * n * (n + 1) + 2.0 * d * n * k
    gram_tf = gram_flops / (ms["prepare"] * 1e-3) / 1e12
    solve_bytes = 4.0 * n * rows_last
    solve_gbs = solve_bytes / (ms["solve"] * 1e-3) / 1e9
    # the prepare call is the operand split (which also forms the column norms), their
    # finalisation and the main product; the figure is for the whole call, the traffic record
    # for the main product kernel
    roof_gram = {"kernel": "gram_dma_kernel", "timed": "nnls_prepare call (presplit_kernel + "
                 "colnorm_finalize_kernel + gram_dma_kernel)", "bound": "mfma",
                 "achieved": round(gram_tf, 2),
                 "peak": round(PEAK_BF16X3_TFLOPS, 1), "unit": "TFLOP/s",
                 "frac": round(gram_tf / PEAK_BF16X3_TFLOPS, 4),
                 "traffic": traffic_record("gram_dma_kernel", "gram.hip")}
    solver = N.solver_name(n, k, N.F32)
    solve_kernel = {"regq": "solve_regq_kernel", "persistent": "solve_persistent_kernel"}.get(
        solver, "solve_" + solver + "_kernel")
    roof_solve = {"kernel": solve_kernel, "bound": "hbm",
                  "achieved": round(solve_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                  "frac": round(solve_gbs / PEAK_HBM_GBS, 4),
                  "traffic": traffic_record(solve_kernel, {"solve_regq_kernel": "solve_regq.hip"}
                                            .get(solve_kernel, "solve_persistent.hip"))}
    dominant, other = ((roof_gram, roof_solve) if ms["prepare"] >= ms["solve"]
                       else (roof_solve, roof_gram))

    out = {
        "metric": "NNLS solves/sec at rel KKT<=1e-5 (plain single RHS); Gram TFLOP/s",
        "value": round(args.steps / wall, 3) if ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3-gram/f32-iter/f64-check",
        "data": "synthetic",
        "config": {"workload": "large single RHS: A 20000x5000 FP32 U[0,1], x 70% zeros Exp(1), "
                               "1% noise, seed 0", "d": d, "n": n, "k": k, "tol": TOL,
                   "parallelism": "single GPU"},
        "roofline": dominant,
        "roofline_other": other,
        "gram_tflops": round(gram_tf, 2),
        "ms": {kk: round(v, 4) for kk, v in ms.items()},
        "solve": {"iters": it_last, "status": st_last, "rows_read": rows_last,
                  "kkt_fp32": float(kkt.cpu()[0])},
        "kkt64_max": float(r64.max()),
        "all_steps_meet_tol": ok,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A_h, b_h, n, it_last, args.cpu_sample_cols)
    print(json.dumps(out), flush=True)


def bench_manyrhs(args):
    """Many right-hand sides sharing A (A 10000 x 256 |N(0,1)|, B = A X + 1 % noise, k = 4096):
    one step = scales + BF16x3 Gram with A^T B + matrix-core many-RHS solve + FP64 refine."""
    import torch
    from paper_1502_01645_amd import nnls as N
    from paper_1502_01645_amd import workloads as W

    dev = torch.device("cuda:0")
    A_h, B_h, _ = W.make_manyrhs()
    d, n = A_h.shape
    k = B_h.shape[1]
    A = torch.from_numpy(A_h).to(dev)
    B = torch.from_numpy(B_h).to(dev)
    s = torch.empty(n, dtype=torch.float64, device=dev)
    Q = torch.empty((n, n), dtype=torch.float32, device=dev)
    q = torch.empty((n, k), dtype=torch.float32, device=dev)
    X = torch.empty((n, k), dtype=torch.float32, device=dev)
    iters = torch.empty(k, dtype=torch.int32, device=dev)
    kkt = torch.empty(k, dtype=torch.float64, device=dev)
    status = torch.empty(k, dtype=torch.int32, device=dev)
    rows = torch.zeros(k, dtype=torch.int64, device=dev)
    kkt64 = torch.empty(k, dtype=torch.float64, device=dev)
    mk = lambda op, mode=0: torch.empty(max(N.workspace_bytes(op, d, n, k, mode, N.F32), 1),  # noqa
                                        dtype=torch.uint8, device=dev)
    ws_p, ws_v, ws_r = mk(N.OP_PREPARE, N.GRAM_BF16X3), mk(N.OP_SOLVE), mk(N.OP_REFINE)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    total = args.warmup + args.steps
    marks = [[ev() for _ in range(4)] for _ in range(total)]

    def step(i):
        e = marks[i]
        e[0].record()
        N.prepare(A, B, N.GRAM_BF16X3, out=(Q, q, s), ws=ws_p)
        e[1].record()
        N.solve(Q, q, s, tol=INNER_TOL, max_iter=5 * n, out=(X, iters, kkt, status), ws=ws_v,
                rows_read=rows)
        e[2].record()
        N.refine(A, B, X, out=(kkt64, None), ws=ws_r)
        e[3].record()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, total):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed = marks[args.warmup:]
    ms = {name: float(np.mean([m[j].elapsed_time(m[j + 1]) for m in timed]))
          for j, name in enumerate(["prepare", "solve", "refine"])}
    r64 = kkt64.cpu().numpy()
    it = iters.cpu().numpy()
    ok = bool(np.all(r64 <= TOL))
    gram_flops = d * n * (n + 1) + 2.0 * d * n * k
    out = {
        "metric": "NNLS solves/sec at rel KKT<=1e-5 (many RHS sharing A)",
        "value": round(k * args.steps / wall, 1) if ok else 0.0,
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3-gram/f32-mfma-iter/f64-check",
        "data": "synthetic",
        "config": {"workload": "many RHS: A 10000x256 |N(0,1)|, X 80% zeros Gamma(2,1), "
                               "B = AX + 1% noise, k=4096, seed 0", "d": d, "n": n, "k": k,
                   "tol": TOL},
        "ms": {kk: round(v, 4) for kk, v in ms.items()},
        "gram_tflops": round(gram_flops / (ms["prepare"] * 1e-3) / 1e12, 2),
        "iters": {"mean": float(it.mean()), "p99": float(np.percentile(it, 99)),
                  "max": int(it.max())},
        "kkt64": {"max": float(r64.max()), "p50": float(np.median(r64)),
                  "p99": float(np.percentile(r64, 99))},
        "all_columns_meet_tol": ok,
    }
    print(json.dumps(out), flush=True)


def bench_ablation(args):
    """The unscaled ablation at full size: the large recipe with lopsided columns (column j
    scaled by 10^u, u ~ U(-1, 1)).  The anti-lopsided path (prepare + solve to the FP32 inner
    tolerance + FP64 check) is timed over the steps; Algorithm 2 on the unscaled (H, h) is then
    run for 1, 10, 100 and 1000 times as many updates as the anti-lopsided solve took, each
    followed by the same FP64 check, which reports the scale-invariant KKT residual of x against
    (A, b) (after its one refinement step, the same for both)."""
    import torch
    from paper_1502_01645_amd import nnls as N
    from paper_1502_01645_amd import workloads as W

    dev = torch.device("cuda:0")
    A_h, b_h, _, _ = W.make_lopsided()
    d, n = A_h.shape
    A = torch.from_numpy(A_h).to(dev)
    b = torch.from_numpy(b_h).to(dev)
    mk = lambda op, mode=0: torch.empty(max(N.workspace_bytes(op, d, n, 1, mode, N.F32), 1),  # noqa
                                        dtype=torch.uint8, device=dev)
    ws_p, ws_g, ws_v, ws_r = mk(N.OP_PREPARE, N.GRAM_BF16X3), mk(N.OP_GRAM, N.GRAM_BF16X3), \
        mk(N.OP_SOLVE), mk(N.OP_REFINE)
    Q = torch.empty((n, n), dtype=torch.float32, device=dev)
    q = torch.empty((n, 1), dtype=torch.float32, device=dev)
    s = torch.empty(n, dtype=torch.float64, device=dev)
    X = torch.empty((n, 1), dtype=torch.float32, device=dev)
    iters = torch.empty(1, dtype=torch.int32, device=dev)
    kkt = torch.empty(1, dtype=torch.float64, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    kkt64 = torch.empty(1, dtype=torch.float64, device=dev)
    obj64 = torch.empty(1, dtype=torch.float64, device=dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    rows = torch.zeros(1, dtype=torch.int64, device=dev)
    marks = [[ev() for _ in range(4)] for _ in range(args.warmup + args.steps)]

    def scaled(i):
        e = marks[i]
        e[0].record()
        N.prepare(A, b, N.GRAM_BF16X3, out=(Q, q, s), ws=ws_p)
        e[1].record()
        N.solve(Q, q, s, tol=INNER_TOL, max_iter=5 * n, out=(X, iters, kkt, status), ws=ws_v,
                rows_read=rows)
        e[2].record()
        N.refine(A, b, X, out=(kkt64, obj64), ws=ws_r)
        e[3].record()

    for i in range(args.warmup):
        scaled(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        scaled(i)
    torch.cuda.synchronize()
    ms_scaled = (time.perf_counter() - t0) * 1e3 / args.steps
    timed = marks[args.warmup:]
    ms = {nm: float(np.mean([mk_[j].elapsed_time(mk_[j + 1]) for mk_ in timed]))
          for j, nm in enumerate(["prepare", "solve", "refine"])}
    m = int(iters.cpu()[0])
    roof = stage_rooflines(N, d, n, 1, ms, int(rows.cpu()[0]))
    r_scaled = float(kkt64.cpu()[0])
    ok = r_scaled <= TOL and int(status.cpu()[0]) == 0

    runs = []
    for mult in (1, 10, 100, 1000):
        e0, e1 = ev(), ev()
        e0.record()
        N.gram(A, b, N.GRAM_BF16X3, out=(Q, q), ws=ws_g)
        N.solve(Q, q, None, tol=0.0, max_iter=mult * m, out=(X, iters, kkt, status), ws=ws_v)
        N.refine(A, b, X, out=(kkt64, obj64), ws=ws_r)
        e1.record()
        torch.cuda.synchronize()
        runs.append({"updates": int(iters.cpu()[0]), "kkt64": float(kkt64.cpu()[0]),
                     "obj64": float(obj64.cpu()[0]), "ms": round(e0.elapsed_time(e1), 3)})
    out = {
        "metric": "NNLS solves/sec at rel KKT<=1e-5 with lopsided columns (anti-lopsided path); "
                  "unscaled Algorithm 2 residual after 1x-1000x the updates",
        "value": round(1e3 / ms_scaled, 3) if ok else 0.0,
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_scaled, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3-gram/f32-iter/f64-check", "data": "synthetic",
        "config": {"workload": "lopsided large single RHS: A 20000x5000 U[0,1] with column j "
                               "scaled by 10^U(-1,1), x 70% zeros Exp(1), 1% noise, seed 0",
                   "d": d, "n": n, "k": 1, "tol": TOL},
        "roofline": roof[0], "roofline_other": roof[1],
        "anti_lopsided": {"updates": m, "kkt64": r_scaled, "ms": round(ms_scaled, 4),
                          "ms_stages": {kk: round(v, 4) for kk, v in ms.items()}},
        "unscaled": runs,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A_h, b_h, n, m, args.cpu_sample_cols)
    print(json.dumps(out), flush=True)


# Mean running time in seconds of the method on each test-case kind, MATLAB on one CPU core
# (Section 5, Table 3); context for the stand-ins, not a target.
PAPER_TABLE3_S = {1: 146.8, 2: 11.9, 3: 71.5, 4: 12.5, 5: 154.7, 6: 12.3}


def bench_paper(args):
    """Stand-ins for the 30 test cases of Section 5 (kinds T1-T6, sparsity 0-40 %, n = 4000,
    d = 6000, b = A x* without noise): each case prepared, solved to the FP32 inner tolerance
    (at most 5 n updates, the paper's cap) and checked in FP64, timed over the steps."""
    import torch
    from paper_1502_01645_amd import nnls as N
    from paper_1502_01645_amd import workloads as W

    dev = torch.device("cuda:0")
    d, n = 6000, 4000
    mk = lambda op, mode=0: torch.empty(max(N.workspace_bytes(op, d, n, 1, mode, N.F32), 1),  # noqa
                                        dtype=torch.uint8, device=dev)
    ws_p, ws_v, ws_r = mk(N.OP_PREPARE, N.GRAM_BF16X3), mk(N.OP_SOLVE), mk(N.OP_REFINE)
    Q = torch.empty((n, n), dtype=torch.float32, device=dev)
    q = torch.empty((n, 1), dtype=torch.float32, device=dev)
    s = torch.empty(n, dtype=torch.float64, device=dev)
    X = torch.empty((n, 1), dtype=torch.float32, device=dev)
    iters = torch.empty(1, dtype=torch.int32, device=dev)
    kkt = torch.empty(1, dtype=torch.float64, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    kkt64 = torch.empty(1, dtype=torch.float64, device=dev)
    obj64 = torch.empty(1, dtype=torch.float64, device=dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    cases, total_ms, total_solves = [], 0.0, 0
    rows = torch.zeros(1, dtype=torch.int64, device=dev)
    stage_ms = {"prepare": 0.0, "solve": 0.0, "refine": 0.0}
    rows_total = 0
    for kind in range(1, 7):
        for sp in W.PAPER_SPARSITY:
            A_h, b_h, _ = W.make_paper_case(kind, sp)
            A = torch.from_numpy(A_h).to(dev)
            b = torch.from_numpy(b_h).to(dev)

            marks = [[ev() for _ in range(4)] for _ in range(args.warmup + args.steps)]

            def one(i):
                e = marks[i]
                e[0].record()
                N.prepare(A, b, N.GRAM_BF16X3, out=(Q, q, s), ws=ws_p)
                e[1].record()
                N.solve(Q, q, s, tol=INNER_TOL, max_iter=5 * n, out=(X, iters, kkt, status),
                        ws=ws_v, rows_read=rows)
                e[2].record()
                N.refine(A, b, X, out=(kkt64, obj64), ws=ws_r)
                e[3].record()

            for i in range(args.warmup):
                one(i)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(args.warmup, args.warmup + args.steps):
                one(i)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            timed = marks[args.warmup:]
            for j, nm in enumerate(["prepare", "solve", "refine"]):
                stage_ms[nm] += float(np.mean([e[j].elapsed_time(e[j + 1]) for e in timed]))
            rows_total += int(rows.cpu()[0])
            total_ms += ms * args.steps
            total_solves += args.steps
            cases.append({"kind": kind, "sparsity": sp, "ms": round(ms, 3),
                          "updates": int(iters.cpu()[0]), "status": int(status.cpu()[0]),
                          "kkt64": float(kkt64.cpu()[0]), "obj64": float(obj64.cpu()[0])})
            del A, b
    ok = all(c["kkt64"] <= TOL for c in cases)
    per_kind = {}
    for kind in range(1, 7):
        cs = [c for c in cases if c["kind"] == kind]
        mean_ms = float(np.mean([c["ms"] for c in cs]))
        per_kind[f"T{kind}"] = {
            "signs_lengths": "/".join(W.PAPER_KINDS[kind]),
            "mean_ms": round(mean_ms, 3),
            "mean_updates": float(np.mean([c["updates"] for c in cs])),
            "max_kkt64": max(c["kkt64"] for c in cs),
            "cases_meeting_tol": sum(c["kkt64"] <= TOL for c in cs),
            "paper_table3_s": PAPER_TABLE3_S[kind],
            "paper_time_over_ours": round(PAPER_TABLE3_S[kind] / (mean_ms * 1e-3), 1),
        }
    out = {
        "metric": "NNLS solves/sec at rel KKT<=1e-5 on stand-ins of the paper's test cases T1-T6",
        "value": round(total_solves / (total_ms * 1e-3), 3) if ok else 0.0,
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total_ms / total_solves, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3-gram/f32-iter/f64-check",
        "data": "synthetic",
        "config": {"workload": "30 stand-ins of Section 5's test cases: kinds T1-T6 (signs +/+-, "
                               "column lengths SAM/RAN/VAR), sparsity 0-40 %, A 6000x4000, "
                               "b = A x* noiseless", "d": d, "n": n, "tol": TOL},
        "per_kind": per_kind,
        "cases": cases,
    }
    # rooflines over the whole set: summed flops / bytes over summed per-case times
    ncase = len(cases)
    roof = stage_rooflines(N, d, n, 1, {kk: v / ncase for kk, v in stage_ms.items()},
                           rows_total / ncase)
    out["roofline"], out["roofline_other"] = roof
    out["ms_stages_mean"] = {kk: round(v / ncase, 4) for kk, v in stage_ms.items()}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        orc = O.load()
        A_h, b_h, _ = W.make_paper_case(3, 0.2)
        t0 = time.perf_counter()
        H, h = orc.gram(A_h, b_h)
        sc, Qo, qo = orc.rescale(H, h)
        _, it_o, _, _ = orc.nqp(Qo, qo[:, 0], TOL, 5 * n)
        t_o = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / t_o, "unit": "solves/s", "cores": orc.num_threads(),
                               "kind": "oracle",
                               "sample": f"one full case (T3, 20 % sparsity, 6000 x 4000): Gram, "
                                         f"rescale and {it_o} updates of Algorithm 2 in FP64, "
                                         f"{t_o:.1f} s"}
    print(json.dumps(out), flush=True)


def bench_nmf(args):
    """Alternating NNLS for a nonnegative factorisation V ~ W H, V 10000 x 4096, rank 256: one
    step = the H half (4096 right-hand sides, matrix W) and the W half (10000 right-hand sides,
    matrix H^T), each prepared, solved on the matrix cores and checked in FP64."""
    import torch
    from paper_1502_01645_amd import nmf as F
    from paper_1502_01645_amd import nnls as N
    from paper_1502_01645_amd import workloads as W

    dev = torch.device("cuda:0")
    V_h, W0_h, _, _ = W.make_nmf()
    m, p = V_h.shape
    r = W0_h.shape[1]
    V = torch.from_numpy(V_h).to(dev)
    alt = F.AlternatingNNLS(V, torch.from_numpy(W0_h).to(dev))
    vnorm2 = float(np.sum(V_h.astype(np.float64) ** 2))
    names = ["H prepare", "H solve", "H check", "H transpose", "W prepare", "W solve", "W check",
             "W transpose"]
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    hist, marks = [], []
    for i in range(args.warmup + args.steps):
        e = [ev() for _ in range(9)]
        alt.step(e)
        torch.cuda.synchronize()
        marks.append(e)
        oh, ow = alt.objective()
        hist.append({"step": i, "rel_residual_after_H": (2 * oh / vnorm2) ** 0.5,
                     "rel_residual_after_W": (2 * ow / vnorm2) ** 0.5, **alt.stats()})
    timed = marks[args.warmup:]
    ms = {nm: float(np.mean([e[j].elapsed_time(e[j + 1]) for e in timed]))
          for j, nm in enumerate(names)}
    ms_step = float(np.mean([e[0].elapsed_time(e[8]) for e in timed]))
    ok = all(h["H"]["kkt64_max"] <= TOL and h["W"]["kkt64_max"] <= TOL for h in hist)
    # matrix-core roofline of the two solves: 2 r flops per row of Q the products read
    rows = sum(h["H"]["rows_read"] + h["W"]["rows_read"] for h in hist[args.warmup:])
    t_solve = float(sum(e[1].elapsed_time(e[2]) + e[5].elapsed_time(e[6]) for e in timed))
    ach = 2.0 * r * rows / (t_solve * 1e-3) / 1e12
    out = {
        "metric": "NNLS column solves/sec in alternating NNLS for NMF (both halves, FP64-checked)",
        "value": round((m + p) * 1e3 / ms_step, 1) if ok else 0.0,
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3-gram/f32-mfma-iter/f64-check", "data": "synthetic",
        "config": {"workload": "NMF by alternating NNLS: V 10000x4096 = max(W* H* + 1% noise, 0), "
                               "W* U[0,1] 30% zeros, H* 70% zeros Exp(1), rank 256, W0 U[0,1]",
                   "m": m, "p": p, "r": r, "tol": TOL},
        "roofline": {"kernel": "solve_mrhs_kernel", "bound": "mfma", "achieved": round(ach, 2),
                     "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": None},
        "ms": {kk: round(v, 4) for kk, v in ms.items()},
        "history": hist,
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        orc = O.load()
        cols = 64
        t0 = time.perf_counter()
        orc.nnls(W0_h, V_h[:, :cols], TOL, 100000)
        t_o = time.perf_counter() - t0
        per_col = t_o / cols
        out["cpu_baseline"] = {
            "value": 1.0 / per_col, "unit": "solves/s", "cores": orc.num_threads(),
            "kind": "oracle",
            "sample": f"oracle Algorithm 1 (Gram, rescale, Algorithm 2 in FP64) on the first "
                      f"{cols} columns of the first H half ({t_o:.2f} s, Gram included)"}
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """Uneven batch (8192 problems, n ~ U{16..512}, d = 3n, A ~ U[0,1], 60 % zeros, 1 % noise):
    one step = one launch of the captured graph plan (batched Gram + queue-driven solves).
    Baseline: the same problems with one nnls_prepare + nnls_solve call pair per problem."""
    import torch
    from oracle import oracle as O
    from paper_1502_01645_amd import nnls as N
    from paper_1502_01645_amd import workloads as W

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    probs = []
    for i in range(args.batch):
        A, b, _ = W.make_batched_problem(i)
        probs.append((A, b[:, 0]))
    t_gen = time.perf_counter() - t0
    A_pool, B_pool, descs = N.pack_problems(probs, dev)
    # the paper's 5 n cap is too tight for the small problems of this batch; cap at 20000
    plan = N.BatchedPlan(A_pool, B_pool, descs, tol=BATCH_INNER_TOL, max_iter=BATCH_MAX_ITER)
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        plan.launch()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_plan = e0.elapsed_time(e1) / args.steps
    st = plan.status.cpu().numpy()
    it = plan.iters.cpu().numpy()
    k32 = plan.kkt.cpu().numpy()
    # FP64 check of a sample against the original data
    X = plan.X_pool.cpu().numpy()
    orc = O.load()
    sample = list(range(0, args.batch, max(1, args.batch // 64)))
    r64 = []
    for i in sample:
        A, b = probs[i]
        dsc = descs[i]
        r, _ = orc.kkt_x(A, b.reshape(-1, 1), X[dsc.offX:dsc.offX + dsc.n].reshape(-1, 1))
        r64.append(r[0])
    r64 = np.array(r64)
    # baseline: one prepare + solve call pair per problem, same kernels family and tolerance
    nmax = max(int(descs[i].n) for i in range(args.batch))
    dmax = max(int(descs[i].d) for i in range(args.batch))
    Qb = torch.empty(nmax * nmax, dtype=torch.float32, device=dev)
    qb = torch.empty(nmax, dtype=torch.float32, device=dev)
    sb = torch.empty(nmax, dtype=torch.float64, device=dev)
    Xb = torch.empty(nmax, dtype=torch.float32, device=dev)
    itb = torch.empty(1, dtype=torch.int32, device=dev)
    kb = torch.empty(1, dtype=torch.float64, device=dev)
    stb = torch.empty(1, dtype=torch.int32, device=dev)
    wsp = torch.empty(N.workspace_bytes(N.OP_PREPARE, dmax, nmax, 1, N.GRAM_BF16X3, N.F32) + 4096,
                      dtype=torch.uint8, device=dev)
    wss = torch.empty(N.workspace_bytes(N.OP_SOLVE, 0, nmax, 1, 0, N.F32) + 4096,
                      dtype=torch.uint8, device=dev)
    nb = min(args.batch, 2048)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nb):
        dsc = descs[i]
        d, n = int(dsc.d), int(dsc.n)
        Ai = A_pool[dsc.offA:dsc.offA + d * n].view(d, n)
        bi = B_pool[dsc.offB:dsc.offB + d].view(d, 1)
        Qi = Qb[:n * n].view(n, n)
        qi = qb[:n].view(n, 1)
        N.prepare(Ai, bi, out=(Qi, qi, sb[:n]), ws=wsp)
        N.solve(Qi, qi, sb[:n], tol=BATCH_INNER_TOL, max_iter=BATCH_MAX_ITER,
                out=(Xb[:n].view(n, 1), itb, kb, stb), ws=wss)
    torch.cuda.synchronize()
    t_base = time.perf_counter() - t0
    base_rate = nb / t_base
    plan_rate = args.batch / (ms_plan * 1e-3)
    sum_flops = sum(float(descs[i].d) * descs[i].n * (descs[i].n + 1) for i in range(args.batch))
    out = {
        "metric": "NNLS solves/sec at rel KKT<=1e-5 (uneven batch, one graph launch)",
        "value": round(plan_rate, 1), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_plan, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3-gram/f32-iter",
        "data": "synthetic",
        "config": {"workload": f"uneven batch: {args.batch} problems, n~U{{16..512}}, d=3n, "
                               "A U[0,1], x 60% zeros U[0,1], 1% noise", "count": args.batch,
                   "tol": TOL, "sum_gram_flop": sum_flops},
        "per_problem_launches": {"value": round(base_rate, 1), "unit": "solves/s",
                                 "problems_timed": nb},
        "speedup_vs_per_problem": round(plan_rate / base_rate, 2),
        "iters": {"mean": float(it.mean()), "max": int(it.max())},
        "all_converged": bool(np.all(st == N.CONVERGED)),
        "status_counts": {str(int(v)): int(c) for v, c in zip(*np.unique(st, return_counts=True))},
        "kkt_fp32_max": float(k32.max()),
        "kkt64_sample": {"count": len(sample), "max": float(r64.max())},
        "gen_s": round(t_gen, 1),
    }
    print(json.dumps(out), flush=True)


def bench_warm(args):
    """Learned warm start (A 4096 x 256 |N(0,1)|, noiseless b = A x, x 85 % zeros Gamma(1.5,1)).
    Training (untimed, reported): the method's own cold solves of 200k seeded right-hand sides,
    then the network trained on them with the library's kernels.  One step = scales + BF16x3
    Gram with A^T B for the 32768 held-out right-hand sides + warm start + many-RHS solve + FP64
    refine; the same step from the cold start is timed beside it."""
    import torch
    from paper_1502_01645_amd import nnls as N
    from paper_1502_01645_amd import workloads as W

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    A_h = W.make_warm_matrix()
    d, n = A_h.shape
    A = torch.from_numpy(A_h).to(dev)
    t0 = time.perf_counter()
    parts = []
    for st in range(0, WARM_TRAIN, 20000):
        Bc, _ = W.make_warm_rhs(A_h, min(20000, WARM_TRAIN - st), split=0, start=st)
        parts.append(torch.from_numpy(Bc).to(dev))
    Btr = torch.cat(parts, 1).contiguous()
    del parts
    Bev_h, _ = W.make_warm_rhs(A_h, WARM_EVAL, split=1, start=0)
    Bev = torch.from_numpy(Bev_h).to(dev)
    log(f"warm: generated {WARM_TRAIN} + {WARM_EVAL} right-hand sides in "
        f"{time.perf_counter() - t0:.1f} s")

    # ---- training set: the method's own solutions, then the network
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    e = [ev() for _ in range(4)]
    e[0].record()
    Qt, qt, _ = N.prepare(A, Btr)
    Ytr, it_tr, _, st_tr = N.solve(Qt, qt, None, WARM_TARGET_TOL, 20000)
    U, T = N.mlp_inputs(qt, Ytr)
    e[1].record()
    del Btr, qt, Ytr
    net = N.WarmStartNet(W.make_mlp_params(0), dev)
    net.fit_input(U)
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    steps_per = WARM_TRAIN // WARM_BATCH
    total = args.epochs * steps_per
    loss = torch.zeros(1, device=dev)
    loss_sum = torch.zeros(1, device=dev)
    step = 0
    e[2].record()
    for ep in range(args.epochs):
        perm = torch.randperm(WARM_TRAIN, device=dev, generator=gen)
        if ep == args.epochs - 1:
            loss_sum.zero_()
        for b in range(steps_per):
            idx = perm[b * WARM_BATCH:(b + 1) * WARM_BATCH]
            lr = WARM_LR * 0.5 * (1.0 + np.cos(np.pi * step / total))
            net.train_step(U[idx].contiguous(), T[idx].contiguous(), lr, WARM_LAMBDA, loss)
            if ep == args.epochs - 1:
                loss_sum += loss
            step += 1
    e[3].record()
    torch.cuda.synchronize()
    train_ms = e[2].elapsed_time(e[3])
    targets_ms = e[0].elapsed_time(e[1])
    train_flop = 3.0 * MLP_FWD_FLOP * WARM_BATCH * total
    log(f"warm: targets {targets_ms:.0f} ms, training {train_ms / 1e3:.1f} s")
    del U, T

    # ---- evaluation: cold and warm steps over the held-out set
    k = WARM_EVAL
    s = torch.empty(n, dtype=torch.float64, device=dev)
    Q = torch.empty((n, n), dtype=torch.float32, device=dev)
    q = torch.empty((n, k), dtype=torch.float32, device=dev)
    X = torch.empty((n, k), dtype=torch.float32, device=dev)
    Y0 = torch.empty((n, k), dtype=torch.float32, device=dev)
    fb = torch.empty(k, dtype=torch.int32, device=dev)
    iters = torch.empty(k, dtype=torch.int32, device=dev)
    kkt = torch.empty(k, dtype=torch.float64, device=dev)
    status = torch.empty(k, dtype=torch.int32, device=dev)
    rows = torch.zeros(k, dtype=torch.int64, device=dev)
    kkt64 = torch.empty(k, dtype=torch.float64, device=dev)
    mk = lambda op, mode=0: torch.empty(max(N.workspace_bytes(op, d, n, k, mode, N.F32), 1),  # noqa
                                        dtype=torch.uint8, device=dev)
    ws_p, ws_v, ws_r = mk(N.OP_PREPARE, N.GRAM_BF16X3), mk(N.OP_SOLVE), mk(N.OP_REFINE)
    total_steps = args.warmup + args.steps
    names = ["prepare", "warm_start", "solve", "refine"]

    def run(warm):
        marks = [[ev() for _ in range(5)] for _ in range(total_steps)]

        def one(i):
            m = marks[i]
            m[0].record()
            N.prepare(A, Bev, N.GRAM_BF16X3, out=(Q, q, s), ws=ws_p)
            m[1].record()
            if warm:
                net.warm_start(Q, q, out=(Y0, fb))
            m[2].record()
            N.solve(Q, q, s, tol=INNER_TOL, max_iter=5 * n, Y0=Y0 if warm else None,
                    out=(X, iters, kkt, status), ws=ws_v, rows_read=rows)
            m[3].record()
            N.refine(A, Bev, X, out=(kkt64, None), ws=ws_r)
            m[4].record()

        for i in range(args.warmup):
            one(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.warmup, total_steps):
            one(i)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        timed = marks[args.warmup:]
        ms = {nm: float(np.mean([m[j].elapsed_time(m[j + 1]) for m in timed]))
              for j, nm in enumerate(names)}
        it = iters.cpu().numpy()
        r64 = kkt64.cpu().numpy()
        res = {"wall": wall, "ms": ms, "iters": it, "r64": r64,
               "status": status.cpu().numpy(), "rows": int(rows.sum().item()),
               "fell_back": float(fb.float().mean().item()) if warm else None}
        return res

    cold = run(False)
    warm = run(True)
    log(f"warm: cold {cold['ms']} warm {warm['ms']}")

    def rate(r):
        return k * args.steps / r["wall"] if bool(np.all(r["r64"] <= TOL)) else 0.0

    v_warm, v_cold = rate(warm), rate(cold)
    ms = warm["ms"]
    # roofline of the dominant kernel of the warm step
    gram_flop = d * n * (n + 1) + 2.0 * d * n * k
    solve_flop = 2.0 * n * warm["rows"]       # algorithmic: rows of Q the products read
    kb = (k + 63) // 64 * 64
    mlp_flop = MLP_FWD_FLOP * kb
    refine_flop = 2.0 * d * n * (n + k) + 3 * 2.0 * n * n * k
    cand = {
        "solve": {"kernel": "solve_mrhs_kernel", "bound": "mfma", "flop": solve_flop,
                  "peak": PEAK_FP32_MFMA_TFLOPS},
        "prepare": {"kernel": "gram_dma_kernel", "bound": "mfma", "flop": gram_flop,
                    "peak": PEAK_BF16X3_TFLOPS},
        "warm_start": {"kernel": "mlp_gemm_kernel", "bound": "mfma", "flop": mlp_flop,
                       "peak": PEAK_BF16_TFLOPS},
        "refine": {"kernel": "gemm_tn_f64_kernel", "bound": "mfma", "flop": refine_flop,
                   "peak": PEAK_FP64_TFLOPS},
    }
    rl = {}
    for nm, c in cand.items():
        ach = c["flop"] / (ms[nm] * 1e-3) / 1e12
        rl[nm] = {"kernel": c["kernel"], "bound": c["bound"], "achieved": round(ach, 2),
                  "peak": round(c["peak"], 1), "unit": "TFLOP/s",
                  "frac": round(ach / c["peak"], 4), "traffic": None}
    dom = max(cand, key=lambda nm: ms[nm])

    def stats(r):
        it = r["iters"]
        return {"solves_per_s": round(rate(r), 1),
                "ms_per_step": round(r["wall"] * 1e3 / args.steps, 3),
                "ms": {kk: round(v, 4) for kk, v in r["ms"].items()},
                "iters_mean": round(float(it.mean()), 2), "iters_p99": float(np.percentile(it, 99)),
                "iters_max": int(it.max()), "kkt64_max": float(r["r64"].max()),
                "all_meet_tol": bool(np.all(r["r64"] <= TOL)),
                "status_counts": {str(int(v)): int(c) for v, c in
                                  zip(*np.unique(r["status"], return_counts=True))}}

    out = {
        "metric": "NNLS solves/sec at rel KKT<=1e-5 (learned warm start, including the network)",
        "value": round(v_warm, 1), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(warm["wall"] * 1e3 / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16-mlp/bf16x3-gram/f32-mfma-iter/f64-check", "data": "synthetic",
        "config": {"workload": f"learned warm start: A {d}x{n} |N(0,1)|, noiseless b = A x, "
                               "x 85% zeros Gamma(1.5,1); trained on 200k method solves, "
                               f"evaluated on {k} held-out", "d": d, "n": n, "k": k, "tol": TOL},
        "roofline": rl[dom],
        "roofline_all": rl,
        "warm": stats(warm),
        "cold": stats(cold),
        "speedup_vs_cold": round(v_warm / v_cold, 3) if v_cold > 0 else None,
        "fallback_rate": warm["fell_back"],
        "training": {"samples": WARM_TRAIN, "epochs": args.epochs, "batch": WARM_BATCH,
                     "lr": WARM_LR, "lambda": WARM_LAMBDA, "target_tol": WARM_TARGET_TOL,
                     "target_solve_ms": round(targets_ms, 1),
                     "target_iters_mean": round(float(it_tr.float().mean().item()), 2),
                     "target_status_nonzero": int((st_tr != 0).sum().item()),
                     "train_s": round(train_ms / 1e3, 2),
                     "train_tflops": round(train_flop / (train_ms * 1e-3) / 1e12, 2),
                     "final_epoch_loss": round(loss_sum.item() / steps_per, 6)},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        orc = O.load()
        m = min(4096, k)
        Bs = np.ascontiguousarray(Bev_h[:, :m], dtype=np.float64)
        t0 = time.perf_counter()
        ito = orc.nnls(A_h.astype(np.float64), Bs, TOL, 0)["iters"]
        t_o = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(m / t_o, 2), "unit": "solves/s", "cores": orc.num_threads(),
            "kind": "oracle",
            "sample": (f"oracle (FP64 Gram, rescale, Algorithm 2 from y = 0) on the first {m} of "
                       f"the {k} held-out right-hand sides: {t_o:.1f} s, mean "
                       f"{float(np.mean(ito)):.1f} iterations; rate = {m} / time")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
