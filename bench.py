"""Benchmarks of the exact sparse products on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2|c1|c3|c4|c5] ...

Default (c2): a step is one product y = A x mod 32749 over the 2,000,000-row
power-law matrix (truncated Zipf(1.8) rows, a 5-diagonal band, 60% of entries
+-1), with A, x and y resident in HBM; block formats are chosen by the trained
selector shipped in the package (--selector heuristic for the plain rules). Prints one JSON line with the roofline
of the product kernel (algorithmic bytes over its HIP-event time against the
8 TB/s HBM peak) and a CPU baseline: the plain C oracle, one thread, on the
host, on repeated full products (checking the GPU result bit for bit).

Other configurations print the same kind of line:
  c1  n = 10,000, 10 per row, m = 65521: A x and A^T x (latency-bound);
  c3  block-Wiedemann sequence U^T A^i V, n = 200,000, s = 8, m = 2^31-1,
      L = 50,003, one hipGraph-replayed fused step per iteration;
  c4  256 uneven matrices with 1..16 right-hand sides, one persistent batched
      launch (tuned) against back-to-back per-matrix launches;
  c5  learned format selection: train on measured block timings, evaluate the
      whole-product time on held-out matrices against the plain heuristic;
  acc the accumulators (int64, fp64, fp32, centered fp32 and fp64) on the
      power-law matrix with m = 4093, times 1, 8 and 16 vectors;
  reorder  a randomly numbered 9-point stencil (2M rows), products in the
      caller's numbering against reverse Cuthill-McKee storage;
  rank the whole block Wiedemann rank of the c3 operand: sequence, order
      basis (PM-Basis), minimal generator, deg det - codeg det.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact nnz·vec/s (bit-exact) + HBM GB/s % peak; learned/batched vs plain"
UNIT = "nnz·vec/s"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["tiles.h", "ffx_impl.h", "k_small.hip", "launch.h", "sg.h", "sg.hip"]  # the one-vector product kernels


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1004_3719_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counters_traffic(name, khash):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if taken on these kernel sources."""
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != khash:
        return None
    return d.get("bytes_per_launch")


def algorithmic_bytes(A, m, vec_bytes=4, s=1):
    """Bytes one product must move in a CSR whose +-1 entries carry no value: 4 B per column index,
    2 B (m < 2^16) or 4 B per other value, 4 B per row pointer, x read once, y written once."""
    r = np.mod(A.val, m)
    n_gen = int(np.count_nonzero((r != 0) & (r != 1) & (r != m - 1)))
    vb = 2 if m < 2**16 else 4
    return 4 * A.nnz + vb * n_gen + 4 * (A.nrows + 1) + vec_bytes * s * (A.ncols + A.nrows)


def line(value, ms, args, dtype, config, roofline, cpu, extra=None, metric=None, unit=None):
    out = {"metric": metric or METRIC, "value": round(value, 1), "unit": unit or UNIT, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config, "roofline": roofline,
           "cpu_baseline": cpu}
    if extra:
        out.update(extra)
    print(json.dumps(out), flush=True)


def event_pairs(n):
    import torch
    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]


def timed(run, steps, stream):
    """(GPU ms per call from one pair of HIP events around `steps` calls on `stream`, wall ms per
    call); the caller has warmed up and synchronized. One pair, not one per call: an event per call
    adds its own few microseconds of GPU time to every call."""
    import torch
    a, b = event_pairs(1)[0]
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(steps):
        run()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps, (time.perf_counter() - t0) * 1e3 / steps


def copy_calibration(mib):
    """A plain elementwise copy (mib MiB read, mib MiB written), three times: the reference
    kernel that scales the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    src = torch.ones(mib * 2**18, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.add(src, 1, out=dst)
    torch.cuda.synchronize()
    del src, dst


def copy_bandwidth(mib=512, reps=5):
    """GB/s of a plain elementwise device copy (mib MiB read + mib MiB written): the achievable
    counterpart of the 8 TB/s peak."""
    import torch
    src = torch.ones(mib * 2**18, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.add(src, 1, out=dst)
    torch.cuda.synchronize()
    a, b = event_pairs(1)[0]
    a.record()
    for _ in range(reps):
        torch.add(src, 1, out=dst)
    b.record()
    torch.cuda.synchronize()
    gbs = 2 * mib * 2**20 * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    return round(gbs, 1)


def pmc_summary(fetch_csv, write_csv, mib, out_path, command):
    """HBM bytes per product launch from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB
    per dispatch), each scaled by what the same counter reads for the calibration copy. The product
    is the 16-bit x copy plus its main kernel (the column-sorted groups, else the tiles)."""
    import csv
    res = {}
    main = None
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        with open(path) as f:
            rows = [r for r in csv.DictReader(f) if r.get("Counter_Name") == counter]
        copy = [float(r["Counter_Value"]) for r in rows if "elementwise" in r["Kernel_Name"]]
        copy = [v for v in copy if v > 0.5 * mib * 1024]
        for name in ("k_sg", "k_tiles"):
            prod = [float(r["Counter_Value"]) for r in rows if name + "<" in r["Kernel_Name"]]
            if prod:
                main = name
                break
        u16 = [float(r["Counter_Value"]) for r in rows if "k_to_u16" in r["Kernel_Name"]]
        if not copy or not prod:
            raise SystemExit("%s: no calibration copy or product dispatch in %s" % (counter, path))
        scale = mib * 1024 / float(np.mean(copy))
        res[counter] = {"copy_kib": round(float(np.mean(copy)), 1), "scale": round(scale, 4),
                        "main_kib": round(float(np.mean(prod)), 1),
                        "k_to_u16_kib": round(float(np.mean(u16)), 1) if u16 else 0.0, "dispatches": len(prod)}
    bpl = sum((v["main_kib"] + v["k_to_u16_kib"]) * 1024 * v["scale"] for v in res.values())
    out = {"kernel": "k_to_u16 + %s, one product of the 2,000,000-row power-law matrix" % main,
           "kernel_hash": kernel_hash(), "counters": res, "bytes_per_launch": int(round(bpl)), "command": command}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def time_oracle(call, seconds, check=None):
    """Repeats an oracle call for at least `seconds`: (calls, seconds, every result passed check)."""
    reps, t, ok = 0, 0.0, True
    while t < seconds or reps < 1:
        t1 = time.perf_counter()
        r = call()
        t += time.perf_counter() - t1
        reps += 1
        if check is not None:
            ok = ok and check(r)
    return reps, t, ok


def omp_threads():
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else len(os.sched_getaffinity(0))


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


# --------------------------------------------------------------------- c2 / c1
def bench_spmv(args, big=True):
    import torch

    import synth
    from paper_1004_3719_amd import Matrix

    dev = torch.device("cuda:0")
    t0 = time.time()
    A = synth.c2() if big else synth.c1()
    m = A.m
    x_np = synth.vector(synth.SEED0 + 1, 1, A.ncols, 0, m - 1)
    log("generated n=%d nnz=%d in %.1fs" % (A.nrows, A.nnz, time.time() - t0))
    t0 = time.time()
    opts = dict(acc=args.acc, selector=args.selector, tile_entries=args.tile_entries, fixed_format=args.fixed_format,
                build_transpose=not big, compact_x=args.compact_x, col_sorted=args.col_sorted)
    if args.selector == "learned":
        opts["model_path"] = args.model
    tuned = None
    if args.tune_tiles:  # the library's tile-size tuner, as a caller keeping this matrix would run it
        from paper_1004_3719_amd.ffx import tune_tile_entries
        topts = {k: v for k, v in opts.items() if k != "tile_entries"}
        best, us = tune_tile_entries(A.nrows, A.ncols, A.rowptr, A.col, A.val, m, s=1, reps=20, **topts)
        opts["tile_entries"] = best
        tuned = {"tile_entries": best, "candidates_us": {str(k): round(v, 2) for k, v in us.items()}}
        log("tile sizes tuned: %s" % tuned)
    M = Matrix.from_synth(A, **opts)
    info = M.info()
    log("built in %.1fs: %s" % (time.time() - t0, info["format_blocks"]))
    x = torch.from_numpy(x_np.astype(np.int32)).to(dev)
    y = torch.empty(A.nrows, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    if args.copy_mib:
        copy_calibration(args.copy_mib)
    for _ in range(args.warmup):
        M.spmv(x, y=y)
    torch.cuda.synchronize()
    kernel_ms, ms = timed(lambda: M.spmv(x, y=y), args.steps, stream)
    log("%d steps: %.4f ms/step wall, %.4f ms/product (events)" % (args.steps, ms, kernel_ms))
    extra = {}
    if not big:
        # a launch-bound product: the same products replayed from a captured HIP graph, which
        # takes the per-call host work (Python, the C ABI, the launch) out of the interval
        want = y.clone()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            M.spmv(x, y=y)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        per_graph = 100
        with torch.cuda.graph(g):
            for _ in range(per_graph):
                M.spmv(x, y=y)
        replays = max(1, args.steps // per_graph)
        g.replay()
        torch.cuda.synchronize()
        graph_ms, _ = timed(g.replay, replays, stream)
        extra["graph_ms_per_product"] = round(graph_ms / per_graph, 5)
        extra["graph_result_equal"] = bool(torch.equal(y, want))
        log("graph replay: %.4f ms/product" % extra["graph_ms_per_product"])
    if not big:  # the plain configuration also times A^T x
        yt = torch.empty(A.ncols, dtype=torch.int32, device=dev)
        for _ in range(args.warmup):
            M.spmv_t(x, y=yt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            M.spmv_t(x, y=yt)
        torch.cuda.synchronize()
        extra["transpose_ms_per_step"] = round((time.perf_counter() - t1) * 1e3 / args.steps, 5)
    b_alg = algorithmic_bytes(A, m)
    achieved = b_alg / (kernel_ms * 1e-3) / 1e9
    main_kernel = "k_sg (column-sorted groups)" if info["sg_groups"] else "k_tiles"
    khash = kernel_hash()
    copy_gbs = copy_bandwidth() if big else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": counters_traffic("spmv_powerlaw_2M_counters.json" if big else "none", khash),
                "kernel": ("k_to_u16 + %s (the product's launches)" % main_kernel
                           if m <= 65536 and (args.compact_x == 1 or (args.compact_x == -1 and A.ncols * 4 > 2**20))
                           else main_kernel),
                "kernel_ms": round(kernel_ms, 5),
                "algorithmic_bytes": int(b_alg),
                "format_bytes": int((info["sg_stream_bytes"] if info["sg_groups"] else info["stream_bytes"])
                                    + 4 * A.ncols + 4 * A.nrows),
                "achievable_copy_GBps": copy_gbs}
    if big:
        # one gather of x per entry: the product's gather rate against the GPU's random-gather rate
        # from a table the size of the gathered x (the 16-bit copy when the product takes one)
        x16 = m <= 65536 and (args.compact_x == 1 or (args.compact_x == -1 and A.ncols * 4 > 2**20))
        row_b = 2 if x16 else 4
        ceil = gather_ceiling(A.ncols * row_b, row_b, A.nnz)
        got = A.nnz / (kernel_ms * 1e-3)
        roofline["gather"] = {"achieved": round(got, 1), "ceiling": round(ceil, 1), "unit": "gathers/s",
                              "frac": round(got / ceil, 4),
                              "ceiling_kernel": "ffx_gather_rate: %d random %d-byte gathers from a %d-byte table"
                                                % (A.nnz, row_b, A.ncols * row_b)}
        if info["sg_groups"]:
            # the column-sorted groups gather 64 consecutive sorted columns per instruction, which span
            # about 64 * ncols * groups / nnz columns: against the same gathers kept inside windows of
            # that many rows (rounded up to a power of two), walked in order as a group walks x
            span = 64.0 * A.ncols * info["sg_groups"] / max(1, A.nnz)
            win = 1 << max(6, int(math.ceil(math.log2(span))))
            ceil_s = gather_ceiling(A.ncols * row_b, row_b, A.nnz, window=win)
            roofline["gather"].update({"ceiling_sorted": round(ceil_s, 1), "frac_sorted": round(got / ceil_s, 4),
                                       "ceiling_sorted_kernel": "ffx_gather_rate: the same gathers inside "
                                                                "%d-row windows visited in order" % win})
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        got = y.cpu().numpy()
        check = lambda want: bool(np.array_equal(got, want))  # noqa: E731
        reps, t_cpu, exact = time_oracle(lambda: oracle.get().spmv(A, x_np), args.cpu_seconds, check)
        reps_a, t_a, exact_a = time_oracle(lambda: oracle.get_all_cores().spmv(A, x_np), args.cpu_seconds / 2, check)
        cpu = {"value": round(A.nnz * reps / t_cpu, 1), "unit": UNIT, "cores": 1, "kind": "oracle",
               "sample": "%d full products y = A x over the same matrix (single thread)" % reps,
               "seconds": round(t_cpu, 2), "gpu_result_bit_exact": exact and exact_a,
               "all_cores": {"value": round(A.nnz * reps_a / t_a, 1), "cores": omp_threads(),
                             "sample": "%d full products, rows over all cores (OpenMP build)" % reps_a,
                             "seconds": round(t_a, 2)},
               "host": host_info()}
        if not (exact and exact_a):
            log("GPU result differs from the oracle")
    workload = ("power-law hybrid SpMV mod 32749: n=2,000,000, truncated Zipf(1.8) rows on [1,5000] + diagonals "
                "-2..2, 60% +-1, x int32") if big else "plain SpMV mod 65521: n=10,000, 10 nnz/row, x int32"
    config = {"workload": workload, "n": A.nrows, "nnz": A.nnz, "m": m, "acc": args.acc, "selector": args.selector,
              "formats": info["format_blocks"], "col_sorted_groups": info["sg_groups"], "kernel_hash": khash}
    if tuned:
        config["tile_tuning"] = tuned
    line(A.nnz / (ms * 1e-3), ms, args, args.acc, config, roofline, cpu, extra)


# ------------------------------------------------------------------ gather
def gather_ceiling(table_bytes, row_bytes, count, window=0):
    """Random gathers per second of the library's calibration kernel (ffx_gather_rate)."""
    from paper_1004_3719_amd.ffx import gather_rate
    return gather_rate(int(table_bytes), int(row_bytes), int(min(count, 2**31 - 1)), int(window), reps=5)


def bench_gather(args):
    """The gather-rate table behind the rooflines: random gathers of 2- to 64-byte rows from tables of
    40 KB to 64 MB, indices streamed coalesced as the products stream their column words, and the same
    gathers kept inside windows of 4,096 rows."""
    import torch
    torch.cuda.init()  # the library's calls run on the device torch initialised
    rows = []
    count = 32 * 2**20
    for row_bytes in (2, 4, 32, 64):
        for table in (40 * 2**10, 2**20, 4 * 2**20, 6553600, 8 * 2**20, 32 * 2**20, 64 * 2**20):
            r = gather_ceiling(table, row_bytes, count)
            rw = gather_ceiling(table, row_bytes, count, window=min(4096, table // row_bytes))
            rows.append({"row_bytes": row_bytes, "table_bytes": table, "gathers_per_s": round(r, 1),
                         "gathers_per_s_window4096": round(rw, 1), "row_GBps": round(r * row_bytes / 1e9, 1)})
            log("rows of %2d B from %9d B: %.1f G/s random, %.1f G/s within 4096-row windows"
                % (row_bytes, table, r / 1e9, rw / 1e9))
    best = max(rows, key=lambda q: q["gathers_per_s"])
    config = {"workload": "random gathers: %d per launch, rows of 2-64 bytes, tables of 40 KB to 64 MB" % count}
    args.steps, args.warmup = len(rows), 0
    line(best["gathers_per_s"], 0.0, args, "u32", config, None, None, {"table": rows}, metric="gathers/s",
         unit="gathers/s")


# ------------------------------------------------------------ accumulators
ACC_NAMES = ["int64", "fp64", "fp32", "fp32c", "fp64c"]


def bench_accumulators(args):
    """The float/double trade-off of the delayed reduction: the power-law matrix with m = 4093, where
    every accumulator applies (fp32 reduces after each term there, centered fp32 after four, the
    others once per row), times 1, 8 and 16 vectors, per accumulator. The line's value is the
    one-vector product of --acc."""
    import torch

    import synth
    from paper_1004_3719_amd import Matrix

    dev = torch.device("cuda:0")
    m = 4093
    A = synth.c2(m=m)
    stream = torch.cuda.current_stream()
    table, ms_main, khash = {}, None, kernel_hash()
    for acc in ACC_NAMES:
        # the tiles for every accumulator (the column-sorted groups are an int64-only path; their
        # one-vector time is the "int64_col_sorted" row)
        M = Matrix.from_synth(A, acc=acc, selector=args.selector, model_path=args.model, col_sorted=0)
        info = M.info()
        row = {"reduce_every": info["reduce_every"]}
        for s_ in (1, 8, 16):
            X = torch.from_numpy(synth.vector(synth.SEED0 + 1, 30 + s_, A.ncols * s_, 0, m - 1)
                                 .astype(np.int32).reshape(A.ncols, s_)).to(dev)
            Y = torch.empty((A.nrows, s_), dtype=torch.int32, device=dev)
            steps = args.steps if s_ == 1 else max(5, args.steps // 8)
            run = (lambda: M.spmv(X[:, 0], y=Y[:, 0])) if s_ == 1 else (lambda: M.spmm(X, Y=Y))
            for _ in range(args.warmup):
                run()
            torch.cuda.synchronize()
            k_ms, _ = timed(run, steps, stream)
            row["s%d_ms" % s_] = round(k_ms, 5)
            row["s%d_Gnnz_vec_per_s" % s_] = round(A.nnz * s_ / (k_ms * 1e-3) / 1e9, 1)
            if s_ == 1 and acc == args.acc:
                ms_main = k_ms
        table[acc] = row
        log("acc %s: %s" % (acc, row))
        M.close()
    M = Matrix.from_synth(A, col_sorted=1)
    x1 = torch.from_numpy(synth.vector(synth.SEED0 + 1, 31, A.ncols, 0, m - 1).astype(np.int32)).to(dev)
    y1 = torch.empty(A.nrows, dtype=torch.int32, device=dev)
    for _ in range(args.warmup):
        M.spmv(x1, y=y1)
    torch.cuda.synchronize()
    k_ms, _ = timed(lambda: M.spmv(x1, y=y1), args.steps, stream)
    table["int64_col_sorted"] = {"s1_ms": round(k_ms, 5), "s1_Gnnz_vec_per_s": round(A.nnz / (k_ms * 1e-3) / 1e9, 1)}
    log("int64, column-sorted groups: %s" % table["int64_col_sorted"])
    M.close()
    b_alg = algorithmic_bytes(A, m)
    achieved = b_alg / (ms_main * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_to_u16 + k_tiles",
                "kernel_ms": round(ms_main, 5), "algorithmic_bytes": int(b_alg)}
    config = {"workload": "accumulator trade-off: the 2,000,000-row power-law matrix with m = 4093 (every "
                          "accumulator applies) times 1, 8 and 16 vectors", "n": A.nrows, "nnz": A.nnz, "m": m,
              "acc": args.acc, "selector": args.selector, "kernel_hash": khash}
    line(A.nnz / (ms_main * 1e-3), ms_main, args, args.acc, config, roofline, None, {"accumulators": table})


# ------------------------------------------------------------- block Wiedemann rank
def bench_rank(args):
    """Block Wiedemann rank of the sequence workload's operand (n = 200,000, 15 entries per row from
    n - 1,000 live columns, m = 2^31 - 1, s = 8): step 1, the sequence S_i = U^T A^i V for i < L =
    50,003 (hipGraph-replayed fused steps); steps 2-3, the order basis of [S(x); -I] (PM-Basis),
    the minimal generator F and rank = deg det F - codeg det F, against the planted rank n - 1,000."""
    import torch

    import synth
    from paper_1004_3719_amd import Matrix, sequence_rank

    dev = torch.device("cuda:0")
    A = synth.c3()
    U_np, V_np = synth.c3_blocks()
    s_ = U_np.shape[1]
    L = synth.c3_length(A.nrows, s_)
    M = Matrix.from_synth(A)
    U, V = torch.from_numpy(U_np).to(dev), torch.from_numpy(V_np).to(dev)
    # warm-up: a short sequence and a small basis
    sequence_rank(M.sequence(U, V, 64), A.m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = M.sequence(U, V, L)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r, D, e, deg = sequence_rank(S, A.m)
    t2 = time.perf_counter()
    planted = A.nrows - 1000
    log("sequence %.3f s, sigma basis + rank %.3f s: rank %d (planted %d), deg det %d, codeg %d"
        % (t1 - t0, t2 - t1, r, planted, D, e))
    ntt_times = {}
    if args.ntt_thresholds:  # steps 2-3 again with other cut-overs to the NTT products
        from paper_1004_3719_amd.ffx import set_ntt_threshold
        for th in (int(v) for v in args.ntt_thresholds.split(",")):
            set_ntt_threshold(th)
            ta = time.perf_counter()
            r2 = sequence_rank(S, A.m)
            ntt_times[th] = round(time.perf_counter() - ta, 4)
            log("NTT above %d coefficients: sigma basis + rank %.3f s, rank %d" % (th, ntt_times[th], r2[0]))
        set_ntt_threshold(1024)
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's order basis, one order at a time, on a bounded prefix of the same sequence
        from oracle import sigma as osig
        Sh = S.cpu().numpy()
        sig = 800  # about 10 s of numpy: the oracle's order basis costs O(sig^2) coefficient products
        t3 = time.perf_counter()
        osig.mbasis(osig.sequence_series(Sh[:sig], A.m), sig, [0] * s_ + [1] * s_, A.m)
        t_cpu = time.perf_counter() - t3
        cpu = {"value": round(sig / t_cpu, 1), "unit": "orders/s", "cores": 1, "kind": "oracle",
               "sample": "order basis of the first %d terms (one order at a time, numpy, single thread)" % sig,
               "seconds": round(t_cpu, 2)}
    total = t2 - t0
    # the dominant kernel is the sequence step: the same per-iteration algorithmic bytes as the
    # sequence workload (A's columns and values and row pointers, W read and written, U read),
    # over the mean time of one iteration of this run's sequence
    b_iter = A.nnz * 8 + 4 * (A.nrows + 1) + 3 * A.nrows * s_ * 8
    it_s = (t1 - t0) / L
    roofline = {"bound": "hbm", "achieved": round(b_iter / it_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(b_iter / it_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_seq_step (sequence; order basis and rank not included)",
                "kernel_ms": round(it_s * 1e3, 5), "algorithmic_bytes": int(b_iter)}
    config = {"workload": "block Wiedemann rank: n=200,000, 15 nnz/row from n-1,000 live columns, m=2^31-1, s=8, "
                          "L=%d; sequence + order basis + generator + rank" % L, "n": A.nrows, "nnz": A.nnz, "L": L,
              "s": s_}
    extra = {"rank": r, "planted_rank": planted, "rank_correct": r == planted, "deg_det": D, "codeg_det": e,
             "generator_degrees": deg, "sequence_s": round(t1 - t0, 3), "sigma_basis_and_rank_s": round(t2 - t1, 3)}
    args.steps, args.warmup = 1, 1
    line(A.nnz * s_ * L / total, total * 1e3, args, "u32 (mod 2^31-1)", config, roofline, cpu, extra)


# ---------------------------------------------------------------- reorder
def bench_reorder(args):
    """A 9-point stencil on a 2048 x 1024 grid whose nodes are numbered at random (2,097,152 rows,
    18.9 M entries, m = 32749): the product in the caller's numbering against the same matrix stored
    in reverse Cuthill-McKee order (one x gather and one y scatter per call), and ten products chained
    through ffx_power, where the permutations are paid once."""
    import torch

    import synth
    from paper_1004_3719_amd import Matrix

    dev = torch.device("cuda:0")
    A = synth.stencil()
    m = A.m
    x_np = synth.vector(synth.SEED0 + 5, 1, A.ncols, 0, m - 1)
    x = torch.from_numpy(x_np.astype(np.int32)).to(dev)
    stream = torch.cuda.current_stream()
    res, y_main = {}, None
    for reorder, cs in ((False, 0), (True, 0), (False, 1), (True, 1)):
        t0 = time.time()
        M = Matrix.from_synth(A, reorder=reorder, selector=args.selector, model_path=args.model, col_sorted=cs)
        build_s = time.time() - t0
        info = M.info()
        y = torch.empty(A.nrows, dtype=torch.int32, device=dev)
        for _ in range(args.warmup):
            M.spmv(x, y=y)
        torch.cuda.synchronize()
        ev_ms, wall_ms = timed(lambda: M.spmv(x, y=y), args.steps, stream)
        a_, b_ = event_pairs(1)[0]
        M.power(10, x)
        a_.record(stream)
        M.power(10, x)
        b_.record(stream)
        torch.cuda.synchronize()
        key = ("reordered" if reorder else "caller_order") + ("_col_sorted" if cs else "_tiles")
        res[key] = {"build_s": round(build_s, 2), "bandwidth": info["bandwidth_stored"], "wall_ms": round(wall_ms, 5),
                    "event_ms": round(ev_ms, 5), "power10_ms_per_product": round(a_.elapsed_time(b_) / 10, 5),
                    "formats": info["format_blocks"], "col_sorted_groups": info["sg_groups"]}
        log("%s: %s" % (key, res[key]))
        if reorder and cs:
            y_main, ms, kernel_ms, sg_info = y, wall_ms, ev_ms, info
        M.close()
    info = sg_info
    b_alg = algorithmic_bytes(A, m)
    achieved = b_alg / (kernel_ms * 1e-3) / 1e9
    main_kernel = "k_sg (column-sorted groups)" if info["sg_groups"] else "k_tiles"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_permute_to_u16 (x gathered into the stored order) + %s (y written through the row map)"
                          % main_kernel,
                "kernel_ms": round(kernel_ms, 5), "algorithmic_bytes": int(b_alg)}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        got = y_main.cpu().numpy()
        reps, t_cpu, exact = 0, 0.0, True
        while t_cpu < args.cpu_seconds or reps < 1:
            t1 = time.perf_counter()
            want = orc.spmv(A, x_np)
            t_cpu += time.perf_counter() - t1
            reps += 1
            exact = exact and bool(np.array_equal(got, want))
        cpu = {"value": round(A.nnz * reps / t_cpu, 1), "unit": UNIT, "cores": 1, "kind": "oracle",
               "sample": "%d full products y = A x in the caller's numbering (single thread)" % reps,
               "seconds": round(t_cpu, 2), "gpu_result_bit_exact": exact}
    config = {"workload": "shuffled 9-point stencil SpMV mod 32749: 2048 x 1024 grid, 2,097,152 rows, nodes numbered "
                          "at random, 60% +-1, x int32; stored in reverse Cuthill-McKee order",
              "n": A.nrows, "nnz": A.nnz, "m": m, "selector": args.selector, "col_sorted_groups": info["sg_groups"]}
    line(A.nnz / (ms * 1e-3), ms, args, "int64", config, roofline, cpu, {"orders": res})


# --------------------------------------------------------------------- gf2
def bench_gf2(args):
    """The power-law matrix taken mod 2 (odd values become 1, even values vanish), times a block of
    32*w vectors over GF(2) packed in w 32-bit words per row."""
    import torch

    import synth
    from paper_1004_3719_amd import Matrix

    dev = torch.device("cuda:0")
    w = args.gf2_words
    A = synth.c2()
    A.m = 2
    M = Matrix.from_synth(A, selector=args.selector)
    info = M.info()
    nnz = info["nnz"]  # entries left after reduction mod 2
    rng = np.random.default_rng(11)
    X_np = rng.integers(-(2**31), 2**31, size=(A.ncols, w), dtype=np.int64).astype(np.int32)
    X = torch.from_numpy(X_np).to(dev)
    Y = torch.empty((A.nrows, w), dtype=torch.int32, device=dev)
    for _ in range(args.warmup):
        M.spmm_gf2(X, Y)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    kernel_ms, ms = timed(lambda: M.spmm_gf2(X, Y), args.steps, stream)
    vecs = 32 * w
    b_alg = 4 * nnz + 4 * (A.nrows + 1) + 4 * w * (A.ncols + A.nrows)  # no values over GF(2)
    achieved = b_alg / (kernel_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": ("k_sg (column-sorted groups, exclusive-or sums)" if w == 1 and M.info()["sg_groups"]
                           else "k_tiles (GF(2) packed)"),
                "kernel_ms": round(kernel_ms, 5), "algorithmic_bytes": int(b_alg)}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        # a bounded sample: the oracle on the first rows and the 32 vectors of the first word, unpacked
        rows = 262144
        sub = synth.rows(synth.c2_spec(), 0, rows)
        sub.m = 2
        Xb = ((X_np[:, 0].view(np.uint32)[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.int64)
        t1 = time.perf_counter()
        Yb = orc.spmm(sub, Xb)
        t_cpu = time.perf_counter() - t1
        packed = (Yb.astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)
        exact = bool(np.array_equal(packed.view(np.int32), Y[:rows, 0].cpu().numpy()))
        sub_nnz = int(np.count_nonzero(np.mod(sub.val, 2)))
        cpu = {"value": round(sub_nnz * 32 / t_cpu, 1), "unit": UNIT, "cores": 1, "kind": "oracle",
               "sample": "the first %d rows times the 32 vectors of the first word, unpacked (single thread)" % rows,
               "seconds": round(t_cpu, 2), "gpu_result_bit_exact": exact}
    config = {"workload": "power-law SpMM over GF(2): the 2,000,000-row power-law matrix mod 2 (%d entries) "
                          "times %d bit-packed vectors (%d words per row)" % (nnz, vecs, w),
              "n": A.nrows, "nnz": nnz, "vectors": vecs, "formats": info["format_blocks"]}
    line(nnz * vecs / (ms * 1e-3), ms, args, "u32 (xor)", config, roofline, cpu)


def bench_gf2_sequence(args):
    """The block-Wiedemann sequence over GF(2): the 200,000-row operand of the sequence workload taken
    mod 2 (every entry 1), 32w packed vectors, L = 2n/(32w) + 3 terms."""
    import torch

    import synth
    from paper_1004_3719_amd import Matrix

    dev = torch.device("cuda:0")
    w = args.gf2_words
    vecs = 32 * w
    A = synth.c3(m=2)
    n = A.nrows
    L = args.seq_length or (2 * n) // vecs + 3
    M = Matrix.from_synth(A)
    rng = np.random.default_rng(12)
    U_np = rng.integers(-(2**31), 2**31, size=(n, w), dtype=np.int64).astype(np.int32)
    V_np = rng.integers(-(2**31), 2**31, size=(n, w), dtype=np.int64).astype(np.int32)
    U, V = torch.from_numpy(U_np).to(dev), torch.from_numpy(V_np).to(dev)
    M.sequence_gf2(U, V, 4)
    torch.cuda.synchronize()
    a, b = event_pairs(1)[0]
    a.record()
    S = M.sequence_gf2(U, V, L)
    b.record()
    torch.cuda.synchronize()
    ev_ms = a.elapsed_time(b)
    nnz = M.info()["nnz"]
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        ub = ((U_np.view(np.uint32)[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(n, -1)
        vb = ((V_np.view(np.uint32)[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(n, -1)
        Lc = 4
        t1 = time.perf_counter()
        So = orc.sequence(A, ub.astype(np.int64), vb.astype(np.int64), Lc)
        t_cpu = time.perf_counter() - t1
        packed = np.stack([(So[i].reshape(vecs, w, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64))
                           .sum(axis=2).astype(np.uint32).view(np.int32) for i in range(Lc)])
        exact = bool(np.array_equal(packed, S[:Lc].cpu().numpy()))
        cpu = {"value": round(nnz * vecs * Lc / t_cpu, 1), "unit": UNIT, "cores": 1, "kind": "oracle",
               "sample": "sequence prefix i = 0..%d at full size, %d unpacked vectors (single thread)" % (Lc - 1, vecs),
               "seconds": round(t_cpu, 2), "gpu_result_bit_exact": exact}
    config = {"workload": "block-Wiedemann sequence over GF(2): n=200,000, 15 nnz/row (all 1), %d packed vectors, "
                          "L=%d" % (vecs, L), "n": n, "nnz": nnz, "vectors": vecs, "L": L}
    args.steps, args.warmup = L, 1
    line(nnz * vecs * L / (ev_ms * 1e-3), ev_ms / L, args, "u32 (xor)", config, None, cpu)


# ---------------------------------------------------------------------- c3
def bench_sequence(args):
    import torch

    import synth
    from paper_1004_3719_amd import Matrix

    dev = torch.device("cuda:0")
    A = synth.c3()
    U, V = synth.c3_blocks()
    L = args.seq_length or synth.c3_length(A.nrows, 8)
    M = Matrix.from_synth(A)
    Ud, Vd = torch.from_numpy(U).to(dev), torch.from_numpy(V).to(dev)
    M.sequence(Ud, Vd, 4)  # warm
    torch.cuda.synchronize()
    a, b = event_pairs(1)[0]
    t0 = time.perf_counter()
    a.record()
    S = M.sequence(Ud, Vd, L)
    b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = a.elapsed_time(b)
    per_iter_ms = ev_ms / L
    work = A.nnz * 8 * L
    # per-iteration bytes: A (col 4 B + val 4 B + row pointers), W read and written, U read
    b_iter = A.nnz * 8 + 4 * (A.nrows + 1) + 3 * A.nrows * 8 * 8
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        t1 = time.perf_counter()
        orc.sequence(A, U, V, 2)  # calibrates the sample length
        per = (time.perf_counter() - t1) / 2
        Lc = int(min(L, max(2, args.cpu_seconds / per)))
        t1 = time.perf_counter()
        So = orc.sequence(A, U, V, Lc)
        t_cpu = time.perf_counter() - t1
        exact = bool(np.array_equal(S[:Lc].cpu().numpy(), So))
        t1 = time.perf_counter()
        So_a = oracle.get_all_cores().sequence(A, U, V, Lc)
        t_a = time.perf_counter() - t1
        exact = exact and bool(np.array_equal(So_a, So))
        cpu = {"value": round(A.nnz * 8 * Lc / t_cpu, 1), "unit": UNIT, "cores": 1, "kind": "oracle",
               "sample": "sequence prefix i = 0..%d at full size (single thread)" % (Lc - 1),
               "seconds": round(t_cpu, 2), "gpu_result_bit_exact": exact,
               "all_cores": {"value": round(A.nnz * 8 * Lc / t_a, 1), "cores": omp_threads(), "seconds": round(t_a, 2),
                             "sample": "the same prefix; the products' rows over all cores (OpenMP build), the "
                                       "projection on one"},
               "host": host_info()}
    roofline = {"bound": "hbm", "achieved": round(b_iter / (per_iter_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(b_iter / (per_iter_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic": None, "kernel": "k_seq_step", "kernel_ms": round(per_iter_ms, 5),
                "algorithmic_bytes": int(b_iter)}
    # the bound that matters: one 32-byte row of W_i (8 int32 residues) gathered per entry, from a table
    # of n * 32 bytes, against the GPU's random row-gather rate from a table of that size
    ceil = gather_ceiling(A.ncols * 32, 32, A.nnz)
    got = A.nnz / (per_iter_ms * 1e-3)
    roofline["gather"] = {"achieved": round(got, 1), "ceiling": round(ceil, 1), "unit": "row gathers/s",
                          "frac": round(got / ceil, 4),
                          "ceiling_kernel": "ffx_gather_rate: random 32-byte rows from a %d-byte table" % (A.ncols * 32)}
    # integer multiply-adds per iteration (product 8 per entry, projection 64 per row), each one
    # v_mad_u64_u32 at a quarter of the 32-bit rate: 256 CUs x 64 lanes x 2.4 GHz / 4
    macs = A.nnz * 8 + A.nrows * 64
    alu_peak = 256 * 64 * 2.4e9 / 4
    roofline["alu"] = {"macs_per_iteration": int(macs), "achieved": round(macs / (per_iter_ms * 1e-3), 1),
                       "peak": alu_peak, "unit": "MAC/s", "frac": round(macs / (per_iter_ms * 1e-3) / alu_peak, 4)}
    config = {"workload": "block-Wiedemann sequence U^T A^i V mod 2^31-1: n=200,000, 15 nnz/row, s=8 int64, "
                          "L=%d" % L, "n": A.nrows, "nnz": A.nnz, "s": 8, "L": L}
    # the same steps launched one per iteration from the host, against the hipGraph replay
    from paper_1004_3719_amd import set_sequence_graph_batch
    Lc = min(L, 4096)
    cmp = {}
    for gb in (64, 0):
        set_sequence_graph_batch(gb)
        M.sequence(Ud, Vd, 4)
        torch.cuda.synchronize()
        a, b = event_pairs(1)[0]
        a.record()
        M.sequence(Ud, Vd, Lc)
        b.record()
        torch.cuda.synchronize()
        cmp["graph_batch_%d" % gb] = round(a.elapsed_time(b) / Lc, 5)
    set_sequence_graph_batch(64)
    args.steps, args.warmup = L, 1
    line(work / (ev_ms * 1e-3), per_iter_ms, args, "int64", config, roofline, cpu,
         {"wall_seconds": round(wall, 3), "ms_per_iteration_%d_iterations" % Lc: cmp})


# ---------------------------------------------------------------------- c4
def bench_batch(args):
    import torch

    import synth
    from paper_1004_3719_amd import Batch, Matrix

    dev = torch.device("cuda:0")
    count = args.batch_count
    t0 = time.time()
    mats, Ms, Xs, Ys, S, work, b_alg = [], [], [], [], [], 0, 0
    for k in range(count):
        A = synth.c4_matrix(k)
        Ms.append(Matrix.from_synth(A))
        Xs.append(torch.from_numpy(synth.c4_rhs(k, A).astype(np.int32)).to(dev))
        Ys.append(torch.empty((A.nrows, A.s), dtype=torch.int32, device=dev))
        S.append(A.s)
        work += A.nnz * A.s
        b_alg += algorithmic_bytes(A, A.m, 4, A.s)
        mats.append(A if k < 64 else None)  # kept for the CPU baseline and the exactness check
    log("built %d matrices in %.1fs, sum nnz*s = %.4g" % (count, time.time() - t0, work))

    def ev_time(f, reps):
        f()
        torch.cuda.synchronize()
        a, b = event_pairs(1)[0]
        a.record()
        for _ in range(reps):
            f()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def per_matrix():
        for M, X, Y in zip(Ms, Xs, Ys):
            M.spmm(X, Y=Y)

    B = Batch(Ms, S)
    if args.skip_compare:  # the batch alone (profiling runs): no per-matrix launches, tuner from its cache
        t_per = t_per_gpu = t_default = float("nan")
    else:
        t_per = ev_time(per_matrix, args.steps)
        # the same launches without host gaps: each matrix timed alone on the GPU, summed
        t_per_gpu = 0.0
        for M, X, Y in zip(Ms, Xs, Ys):
            t_per_gpu += ev_time(lambda: M.spmm(X, Y=Y), 3)
        t_default = ev_time(lambda: B.spmm(Xs, Ys), args.steps)
    best = B.tune(Xs, Ys, reps=3, cache_path=args.tune_cache or None)
    t_batch = ev_time(lambda: B.spmm(Xs, Ys), args.steps)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        t_cpu, w_cpu, exact = 0.0, 0, True
        for k, A in enumerate(mats):
            if A is None or (t_cpu >= args.cpu_seconds and k >= 8):
                break
            t1 = time.perf_counter()
            want = orc.spmm(A, synth.c4_rhs(k, A))
            t_cpu += time.perf_counter() - t1
            w_cpu += A.nnz * A.s
            exact = exact and bool(np.array_equal(Ys[k].cpu().numpy(), want))
        nk = k + 1
        # all cores, on the same leading matrices (the batch's other matrices were not kept on the host)
        orc_a = oracle.get_all_cores()
        t_a, w_a = 0.0, 0
        for k, A in enumerate(mats[:nk]):
            t1 = time.perf_counter()
            orc_a.spmm(A, synth.c4_rhs(k, A))
            t_a += time.perf_counter() - t1
            w_a += A.nnz * A.s
        cpu = {"value": round(w_cpu / t_cpu, 1), "unit": UNIT, "cores": 1, "kind": "oracle",
               "sample": "the first %d matrices of the batch, all right-hand sides (single thread)" % nk,
               "seconds": round(t_cpu, 2), "gpu_result_bit_exact": exact,
               "all_cores": {"value": round(w_a / t_a, 1), "cores": omp_threads(), "seconds": round(t_a, 2),
                             "sample": "the same matrices, rows over all cores (OpenMP build)"},
               "host": host_info()}
    config = {"workload": "256 uneven matrices mod 65521, n log-uniform [2000, 500000], 3..60 nnz/row, "
                          "uniform/banded/block-diagonal, 70% +-1, 1..16 int32 right-hand sides",
              "count": count, "sum_nnz_times_s": work, "tuned": best}
    extra = {"per_matrix_ms": round(t_per, 4), "per_matrix_gpu_sum_ms": round(t_per_gpu, 4),
             "batch_untuned_ms": round(t_default, 4), "batch_speedup_vs_per_matrix": round(t_per / t_batch, 3),
             "batch_speedup_vs_per_matrix_gpu_sum": round(t_per_gpu / t_batch, 3)}
    achieved = b_alg / (t_batch * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_batch (persistent)",
                "kernel_ms": round(t_batch, 5), "algorithmic_bytes": int(b_alg)}
    # one row gather of X per entry and column chunk (at most 8 columns, 32 bytes). The ceiling adds,
    # matrix by matrix, the time the calibration kernel takes for that many gathers of rows of the
    # chunk's width (rounded up to a power of two) from a table of the X block's size (likewise):
    # uniformly
    # random for the uniform-column matrices, inside 4,096-row windows for the banded and
    # block-diagonal ones
    rates, t_ceil, nnz_chunks = {}, 0.0, 0
    for k in range(count):
        nnz_k = Ms[k].info()["nnz"]
        chunks = (S[k] + 7) // 8
        row_bytes = 1 << int(math.ceil(math.log2(4 * min(S[k], 8))))  # the calibration's widths: powers of 2
        table = 1 << max(13, int(math.ceil(math.log2(max(1, Ms[k].info()["ncols"] * S[k] * 4)))))
        window = 0 if synth.c4_params(k)["structure"] == 0 else 4096
        key = (table, row_bytes, window)
        if key not in rates:
            rates[key] = gather_ceiling(table, row_bytes, 8 * 2**20, window=min(window, table // row_bytes))
        t_ceil += nnz_k * chunks / rates[key]
        nnz_chunks += nnz_k * chunks
    ceil = nnz_chunks / t_ceil
    got = nnz_chunks / (t_batch * 1e-3)
    roofline["gather"] = {"achieved": round(got, 1), "ceiling": round(ceil, 1), "unit": "row gathers/s",
                          "frac": round(got / ceil, 4), "ceiling_calibrations": len(rates),
                          "ceiling_kernel": "ffx_gather_rate per matrix: rows of the chunk's width from a table of "
                                            "its X block's size, random (uniform columns) or in 4,096-row windows"}
    line(work / (t_batch * 1e-3), t_batch, args, "int64", config, roofline, cpu, extra)


# ---------------------------------------------------------------------- c5
def bench_selector(args):
    import torch

    import synth
    from paper_1004_3719_amd import selector_train as ST
    from paper_1004_3719_amd.ffx import FORMATS

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(args.seed)
    BR = 4096
    if args.labels and os.path.exists(args.labels):
        with np.load(args.labels) as z:
            X, T, H = z["X"], z["T"], z["H"]
        log("loaded %d labelled blocks from %s" % (len(X), args.labels))
    else:
        Xs, Ts, Hs = [], [], []
        t0 = time.time()
        for k in range(args.train_mats):
            sp, p = synth.c5_spec(k)
            nb = max(1, sp.nrows // BR)
            b0 = int(rng.integers(0, max(1, nb - args.train_blocks + 1)))
            r0, r1 = b0 * BR, min(sp.nrows, (b0 + args.train_blocks) * BR)
            A = ST.shift_columns(synth.rows(sp, r0, r1), r0)
            A.m = synth.M_C5
            F, T, H = ST.window_labels(A, seed=k)
            Xs.append(F)
            Ts.append(T)
            Hs.append(H)
            if k % 20 == 19:
                log("labels: %d matrices, %d blocks, %.0fs" % (k + 1, sum(len(f) for f in Xs), time.time() - t0))
        X = np.concatenate(Xs)
        T = np.concatenate(Ts)
        H = np.concatenate(Hs)
        if args.labels:
            np.savez(args.labels, X=X, T=T, H=H)
    log("training on %d blocks" % len(X))
    nval = max(1, len(X) // 10)
    model = args.model_out
    os.makedirs(os.path.dirname(model), exist_ok=True)
    S, rep = ST.train(X, T, H, epochs=args.epochs, lr=args.lr, seed=args.seed, n_val=nval, out_model=model)
    mu = rep["margin"]
    hist = [{"train_loss": rep["train_loss"], "val_loss": rep["val_loss"], "steps": rep["steps"]}]
    log("trained in the library: %s" % json.dumps(rep))
    # held-out blocks: summed block time of each choice relative to the best per block
    learned, _ = ST.choose(S, X[:nval])
    block_cost = {"learned": round(ST.choice_cost(T[:nval], learned), 4),
                  "heuristic": round(ST.choice_cost(T[:nval], H[:nval]), 4)}
    for f, name in enumerate(FORMATS):
        block_cost["all_" + name] = round(ST.choice_cost(T[:nval], np.full(nval, f)), 4)
    log("validation blocks, summed time / best: %s" % json.dumps(block_cost))
    # held-out matrices: whole-product time of the learned formats, the heuristic's and each format forced
    # on every block (medians of 3 interleaved rounds); every product checked against the oracle
    import oracle
    orc = oracle.get()
    tot = {}
    same, nev = True, 0
    eval_fixed = FORMATS if args.eval_fixed == "all" else [f for f in args.eval_fixed.split(",") if f]
    for f in eval_fixed:
        if f not in FORMATS:
            raise SystemExit("--eval-fixed: unknown format %s (formats: %s)" % (f, ",".join(FORMATS)))
    for k in range(1800, 1800 + args.eval_mats):
        sp, p = synth.c5_spec(k)
        r1 = min(sp.nrows, args.eval_rows) if args.eval_rows else sp.nrows
        A = synth.rows(sp, 0, r1)
        A.m = synth.M_C5
        xh = synth.vector(k, 8, A.ncols, 0, A.m - 1)
        x = torch.from_numpy(xh.astype(np.int32)).to(dev)
        r = ST.evaluate(A, model, x, reps=10, fixed=eval_fixed, rounds=3)
        want = orc.spmv(A, xh)
        for y in r["results"].values():
            same = same and np.array_equal(y.cpu().numpy(), want)
        for key, v in r.items():
            if key.endswith("_us"):
                tot[key] = tot.get(key, 0.0) + v
        nev += 1
        if nev % 10 == 0 or not args.eval_rows:
            log("held-out %d (matrix %d, %d rows, %d entries): totals so far %s, equal to the oracle %s"
                % (nev, k, A.nrows, A.nnz, json.dumps({key: round(v, 1) for key, v in tot.items()}), same))
    if not nev:  # training only (--eval-mats 0)
        print(json.dumps({"trained": rep, "validation_block_cost_vs_best": block_cost, "model": model}), flush=True)
        return
    tot_h, tot_l = tot["heuristic_us"], tot["learned_us"]
    fixed = {f: tot["fixed_%s_us" % f] for f in eval_fixed}
    best_fixed = min(fixed, key=fixed.get) if fixed else None
    log("held-out: heuristic %.1f us, learned %.1f us, best fixed %s %.1f us, all equal to the oracle %s"
        % (tot_h, tot_l, best_fixed, fixed.get(best_fixed, float("nan")), same))
    config = {"workload": "learned format selection mod 65521: %d training windows x %d blocks, %d held-out "
                          "matrices (%s), 32->64->64->6 FP32"
                          % (args.train_mats, args.train_blocks, nev,
                             "first %d rows each" % args.eval_rows if args.eval_rows else "whole"),
              "train_blocks": int(len(X)), "history": hist[-1:]}
    extra = {"validation_block_cost_vs_best": block_cost, "decision_margin_log2": mu,
             "heuristic_total_us": round(tot_h, 1), "learned_total_us": round(tot_l, 1),
             "fixed_total_us": {f: round(v, 1) for f, v in fixed.items()}, "best_fixed_format": best_fixed,
             "learned_speedup_vs_heuristic": round(tot_h / max(tot_l, 1e-9), 4),
             "learned_speedup_vs_best_fixed": round(fixed[best_fixed] / max(tot_l, 1e-9), 4) if fixed else None,
             "timing": "per matrix: median of 3 interleaved rounds of 10 launches",
             "results_equal_oracle": same}
    args.steps, args.warmup = nev, 0
    line(0.0, tot_l / 1e3, args, "fp32 network / int64 products", config, None, None, extra)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "gf2", "gf2seq", "acc", "reorder", "rank",
                                                      "gather"])
    ap.add_argument("--gf2-words", type=int, default=8, help="32-bit words per row in the GF(2) product")
    ap.add_argument("--acc", default="int64", choices=ACC_NAMES)
    ap.add_argument("--selector", default="learned", choices=["heuristic", "learned"],
                    help="block format chooser: the trained network shipped in the package (falls back to the "
                         "heuristic if the model is missing) or the plain heuristic")
    ap.add_argument("--model", default=os.path.join(ROOT, "paper_1004_3719_amd", "models", "selector.bin"))
    ap.add_argument("--tile-entries", type=int, default=0)
    ap.add_argument("--ntt-thresholds", default="",
                    help="rank: also time steps 2-3 with these NTT cut-overs (comma list of lengths)")
    ap.add_argument("--tune-tiles", action="store_true",
                    help="c1/c2: pick tile_entries with the library's tuner (ffx_tune_tile_entries) before building")
    ap.add_argument("--compact-x", type=int, default=-1, choices=[-1, 0, 1],
                    help="16-bit copy of x for m <= 65536: -1 auto (x above 1 MiB), 0 never, 1 always")
    ap.add_argument("--fixed-format", default=None)
    ap.add_argument("--col-sorted", type=int, default=-1, choices=[-1, 0, 1],
                    help="column-sorted row groups for the one-vector product: -1 auto, 0 never, 1 always")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seq-length", type=int, default=0)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--tune-cache", default="", help="JSON cache of the batch tuner (read if it holds this batch)")
    ap.add_argument("--skip-compare", action="store_true", help="batch: skip the per-matrix comparison launches")
    ap.add_argument("--train-mats", type=int, default=600)
    ap.add_argument("--train-blocks", type=int, default=16)
    ap.add_argument("--eval-mats", type=int, default=200)
    ap.add_argument("--eval-rows", type=int, default=131072, help="rows of each held-out matrix (0: whole)")
    ap.add_argument("--eval-fixed", default="all",
                    help="held-out matrices: formats forced on every block to compare with (comma list, or all)")
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--labels", default="", help="npz of (features, log2 us) block labels: loaded if present, "
                                                  "else measured and saved there")
    ap.add_argument("--model-out", default=os.path.join(ROOT, "paper_1004_3719_amd", "models", "selector.bin"))
    ap.add_argument("--copy-mib", type=int, default=0, help="run a calibration copy of this size first (counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary of two rocprofv3 --pmc runs and exit (no GPU)")
    ap.add_argument("--pmc-mib", type=int, default=512)
    ap.add_argument("--pmc-command", default="")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.pmc_mib,
                    os.path.join(ROOT, "profiles", "spmv_powerlaw_2M_counters.json"), args.pmc_command)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.config == "c2":
        bench_spmv(args, big=True)
    elif args.config == "c1":
        bench_spmv(args, big=False)
    elif args.config == "c3":
        bench_sequence(args)
    elif args.config == "gf2":
        bench_gf2(args)
    elif args.config == "gf2seq":
        bench_gf2_sequence(args)
    elif args.config == "acc":
        bench_accumulators(args)
    elif args.config == "reorder":
        bench_reorder(args)
    elif args.config == "rank":
        bench_rank(args)
    elif args.config == "gather":
        bench_gather(args)
    elif args.config == "c4":
        args.steps = min(args.steps, 10)
        bench_batch(args)
    else:
        bench_selector(args)


if __name__ == "__main__":
    main()
