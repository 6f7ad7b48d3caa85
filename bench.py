"""Benchmark: batched Shaped 2D-SSA decompositions + reconstructions per second.

Workload (default): the 2D-SSA image workload -- 512x512 images, each a sum of
three planar cosines (periods 8..64 px, random directions) plus N(0, 0.2^2)
noise, window 64x64, r = 30 eigentriples, reconstruction of the groups
{1,2}, {3,4}, {5,6} (0-based {0,1}, {2,3}, {4,5}).  A step decomposes and
reconstructs one batch of B images already resident in device memory.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--batch 64] [--precision fp32]

Prints one JSON line.  Besides the headline rate it reports the plain
single-instance FP64 path on the same GPU, the roofline of the dominant
kernel (HIP-event timing of its launches inside the timed region) and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle sample")
    ap.add_argument("--no-single", action="store_true", help="skip the single-instance FP64 comparator")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the w-correlation, forecast, continuation and eigen-method timings")
    # The serving section is off unless asked for: a full run of it on the
    # build with the FP32 basis copy ended with a GPU memory fault whose cause
    # is not found (see the serving tests' skip reason).
    ap.add_argument("--serve", type=int, default=0, metavar="N",
                    help="requests of the mixed serving workload for the latency runs (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (torch) and exit: the reference "
                         "kernel for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
              "described, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1309_5050_amd as S
    from paper_1309_5050_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        # a plain device copy of known size; the source is evicted from the
        # caches first (512 MiB written after it), so the copy reads HBM
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        flush = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del flush
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))
        return
    stream = torch.cuda.current_stream()
    ctx = S.Context(0, stream=stream.cuda_stream)

    B = args.batch
    n, lw, r = 512, 64, 30
    groups = [[0, 1], [2, 3], [4, 5]]
    imgs = [W.image_2d(n=n, lw=lw, r=r, seed=1000 + i)["x"] for i in range(B)]
    xs = [torch.tensor(x, device=dev) for x in imgs]
    outs = [torch.empty((len(groups), n, n), dtype=torch.float64, device=dev) for _ in range(B)]

    def step(prec):
        ds = ctx.decompose_batch_dev(xs, (lw, lw), r, precision=prec)
        bad = [d for d in ds if isinstance(d, Exception)]
        if bad:
            raise bad[0]
        S.Context.reconstruct_batch_dev(ds, groups, outs)
        return ds

    for _ in range(args.warmup):
        ds = step(args.precision)
        del ds
    torch.cuda.synchronize()
    # HIP events bracket one launch in every PROFILE_EVERY of each timed class
    # (an odd period samples both directions of the column pass); each
    # bracketed launch costs the stream two event records
    ctx.profile(",".join(list(KERNELS) + ["lz_ritz"]), every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        last = None          # a step's results are released before the next step
        last = step(args.precision)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read(list(KERNELS) + ["lz_ritz"])
    ctx.profile(None)
    stats = last[0].stats
    dt = t1 - t0
    value = B * args.steps / dt

    # rooflines of the two product kernels; the dominant one (more time in
    # the timed region) is the headline
    roofs = {}
    for cls, name in KERNELS.items():
        p = prof[cls]
        kern_ms = p["ms"] / max(p["launches"], 1)
        kern_bytes = p["bytes"] / max(p["launches"], 1)
        achieved = kern_bytes / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else 0.0
        traffic, traffic_kernel = measured_traffic(name)
        roofs[cls] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": name,
                      "ms_per_launch": kern_ms, "bytes_per_launch": kern_bytes, "launches": p["launches"],
                      "ms_total": p["ms"], "timed_every": PROFILE_EVERY, "traffic_counters_on": traffic_kernel}
    dominant = max(roofs, key=lambda c: roofs[c]["ms_total"])
    # the matrix-core kernel (FP64 Ritz rotation): its timing class counts
    # floating-point operations
    pr = prof["lz_ritz"]
    mfma = None
    if pr["launches"] > 0 and pr["ms"] > 0:
        tf = pr["bytes"] / (pr["ms"] * 1e-3) / 1e12
        mfma = {"kernel": "k_lz_ritz", "dtype": "f64", "achieved": tf, "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": tf / FP64_MFMA_PEAK_TFLOPS, "launches": pr["launches"],
                "ms_per_launch": pr["ms"] / pr["launches"], "flop_per_launch": pr["bytes"] / pr["launches"]}
    # HbH product rate over the whole product (algorithmic bytes per product)
    L, K = lw * lw, (n - lw + 1) ** 2
    b = 4 if args.precision == "fp32" else 8
    bmv = b * (K + L) + 2 * b * n * (n // 2 + 1)
    products = 2 * sum(d.stats["steps"] for d in last)

    def run_extras():
        """The calls outside the timed batches (w-correlations, forecasts,
        continuation, eigen method), each timed on its own."""
        # w-correlation matrix of the r elementary components of one decomposition
        # (reconstruction of r singleton groups + the weighted Gram kernel)
        ctx.profile("wgram")
        torch.cuda.synchronize()
        tw0 = time.perf_counter()
        rho, _ = last[0].wcor([[i] for i in range(r)])
        tw1 = time.perf_counter()
        pw = ctx.profile_read(["wgram"])["wgram"]
        ctx.profile(None)
        wgram_gbs = pw["bytes"] / (pw["ms"] * 1e-3) / 1e9 if pw["ms"] > 0 else 0.0
        wcor = {"groups": r, "ms_total": 1e3 * (tw1 - tw0), "gram_kernel_ms": pw["ms"],
                "gram_roofline": {"bound": "hbm", "achieved": wgram_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": wgram_gbs / HBM_PEAK_GBS, "bytes": pw["bytes"]},
                "max_offdiag_abs_rho": float(np.max(np.abs(rho - np.diag(np.diag(rho)))))}

        # column recurrent forecast: 100 values of each of the 50 series of the
        # MSSA workload (N_p ~ U(1000, 3000), L = 500, r = 20) from the group of
        # the two shared sines, on an FP32 decomposition
        wm = W.config(3)
        dm = ctx.decompose_multi(wm["x"], wm["window"], wm["r"], precision="fp32")
        torch.cuda.synchronize()
        tf0 = time.perf_counter()
        fc = dm.rforecast([0, 1, 2, 3], 100)
        tf1 = time.perf_counter()
        fv = dm.vforecast([0, 1, 2, 3], 100)
        tf2 = time.perf_counter()
        fr = dm.rforecast([0, 1, 2, 3], 100, direction="row")
        tf3 = time.perf_counter()
        fw = dm.vforecast([0, 1, 2, 3], 100, direction="row")
        tf4 = time.perf_counter()
        rforecast = {"workload": "MSSA 50 series N~U(1000,3000), L=500, r=20, fp32; group {1..4}, 100 steps",
                     "series": int(fc.shape[0]), "steps": int(fc.shape[1]), "ms": 1e3 * (tf1 - tf0),
                     "vector_ms": 1e3 * (tf2 - tf1), "row_ms": 1e3 * (tf3 - tf2), "vector_row_ms": 1e3 * (tf4 - tf3),
                     "finite": bool(np.isfinite(fv).all() and np.isfinite(fr).all() and np.isfinite(fw).all())}
        dm.free()

        # continuation: one decomposition of the workload (FP32) extended by
        # r/5 triplets, against decomposing it afresh with that many
        r2 = r + max(1, r // 5)
        torch.cuda.synchronize()
        te0 = time.perf_counter()
        prec = args.precision
        de = ctx.decompose_batch_dev(xs[:1], (lw, lw), r, precision=prec)[0]
        _ = de.sigma
        te1 = time.perf_counter()
        de.extend(r2)
        _ = de.sigma
        te2 = time.perf_counter()
        df = ctx.decompose_batch_dev(xs[:1], (lw, lw), r2, precision=prec)[0]
        _ = df.sigma
        te3 = time.perf_counter()
        extend = {"workload": f"one {n}x{n} image, {lw}x{lw} window, {prec}", "r_from": r, "r_to": r2,
                  "decompose_ms": 1e3 * (te1 - te0), "extend_ms": 1e3 * (te2 - te1),
                  "fresh_decompose_ms": 1e3 * (te3 - te2),
                  "max_sigma_diff_over_s1": float(np.max(np.abs(de.sigma - df.sigma)) / df.sigma[0])}
        de.free()
        df.free()

        # eigen method against the truncated SVD on a small window: a 1D series
        # of 10000 values with L = 100, r = 10 (FP64 both)
        xe = W.series_1d(n=10000, L=100, r=10)["x"]
        ctx.profile("xgram")
        torch.cuda.synchronize()
        tq0 = time.perf_counter()
        dq = ctx.decompose(xe, 100, 10, method="eigen")
        _ = dq.sigma
        tq1 = time.perf_counter()
        dl = ctx.decompose(xe, 100, 10)
        _ = dl.sigma
        tq2 = time.perf_counter()
        pg = ctx.profile_read(["xgram"])["xgram"]
        ctx.profile(None)
        # the "bytes" of the xgram class count floating-point operations
        xg_tf = pg["bytes"] / (pg["ms"] * 1e-3) / 1e12 if pg["launches"] and pg["ms"] > 0 else None
        eigen = {"workload": "1D series N=10000, L=100, r=10, fp64", "eigen_ms": 1e3 * (tq1 - tq0),
                 "lanczos_ms": 1e3 * (tq2 - tq1),
                 "max_sigma_diff_over_s1": float(np.max(np.abs(dq.sigma - dl.sigma)) / dl.sigma[0]),
                 "xgram_kernel_ms": pg["ms"] / pg["launches"] if pg["launches"] else None,
                 "xgram_tflops": xg_tf,
                 "xgram_mfma_frac": xg_tf / FP64_MFMA_PEAK_TFLOPS if xg_tf else None}
        dq.free()
        dl.free()
        return wcor, rforecast, extend, eigen

    wcor = rforecast = extend = eigen = None
    if not args.no_extras:
        wcor, rforecast, extend, eigen = run_extras()

    # plain single-instance FP64 path (same kernels, batch of one)
    single = None
    if not args.no_single:
        reps = 2
        torch.cuda.synchronize()
        lat = []
        for i in range(reps):
            ta = time.perf_counter()
            d = ctx.decompose_batch_dev(xs[i:i + 1], (lw, lw), r, precision="fp64")[0]
            S.Context.reconstruct_batch_dev([d], groups, outs[i:i + 1])
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - ta)
        single = {"decomps_per_s": reps / sum(lat), "latency_ms": 1e3 * float(np.median(lat))}


    serving = None
    if args.serve > 0:
        serving = serve_bench(S, W, args.serve)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(imgs[0], lw)

    line = {
        "metric": "SSA decomps/s (decompose r=30 + reconstruct 3 groups), 512x512 image, 64x64 window",
        "value": value,
        "unit": "decomps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "2D-SSA 512x512 image, 64x64 window, r=30, groups {1,2},{3,4},{5,6}",
                   "batch": B, "precision": args.precision + (" products, fp64 Lanczos" if
                                                             args.precision == "fp32" else ""),
                   "parallelism": "batched on 1 GPU"},
        "roofline": roofs[dominant],
        "roofline_kernels": roofs,
        "mfma": mfma,
        "wcor": wcor,
        "rforecast": rforecast,
        "extend": extend,
        "eigen": eigen,
        "hbh_product": {"bytes_per_product": bmv, "products_per_step": products,
                        "effective_GBs": bmv * products / (dt / args.steps) / 1e9},
        "lanczos": {"steps": stats["steps"], "restarts": stats["restarts"], "basis": stats["basis"],
                    "max_resid_over_sigma1": stats["max_resid"]},
        "host_ms_per_batch": {"setup": B * stats["ms_setup"], "lanczos": B * stats["ms_lanczos"],
                              "finish": B * stats["ms_finish"]},
        "fp64_single_instance": single,
        "speedup_vs_fp64_single": (value / single["decomps_per_s"]) if single else None,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


def _run_sync(ctx, q, prec):
    if q["kind"] == "mssa":
        d = ctx.decompose_multi(q["x"], q["window"], q["r"], precision=prec)
    else:
        d = ctx.decompose(q["x"], q["window"], q["r"], mask=q.get("mask"), wmask=q.get("wmask"), precision=prec)
    d.reconstruct(q["groups"])
    d.free()


def _submit(ctx, q, prec):
    if q["kind"] == "mssa":
        return ctx.submit_multi(q["x"], q["window"], q["r"], precision=prec, groups=q["groups"])
    return ctx.submit(q["x"], q["window"], q["r"], mask=q.get("mask"), wmask=q.get("wmask"), precision=prec,
                      groups=q["groups"])


def _served_run(S, data, prec, rate, seed):
    """Poisson arrivals at `rate` req/s (rate None: all at once, closed loop);
    returns latency percentiles (first 5% excluded) and throughput."""
    import threading

    import numpy as np
    ctx = S.Context(0)
    n = len(data)
    rng = np.random.default_rng(seed)
    arrive = np.cumsum(rng.exponential(1.0 / rate, n)) if rate else np.zeros(n)
    tickets = [None] * n
    lat = [None] * n
    errors = []
    got = threading.Event()

    def collect():
        try:
            for i in range(n):
                while tickets[i] is None:
                    got.wait(0.001)
                ctx.wait(tickets[i])
                d, _, tm = ctx.take(tickets[i])
                lat[i] = tm["total_ms"]
                if hasattr(d, "free"):
                    d.free()
                else:
                    errors.append(f"request {i}: {d!r}")   # a failed request's error
        except Exception as e:   # reported by the main thread
            errors.append(f"collector: {e!r}")

    th = threading.Thread(target=collect)
    th.start()
    t0 = time.perf_counter()
    for i, q in enumerate(data):
        dt = t0 + arrive[i] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tickets[i] = _submit(ctx, q, prec)
        got.set()
    th.join()
    t1 = time.perf_counter()
    ctx.close()
    if errors:
        raise RuntimeError(f"{len(errors)} served requests failed ({prec}); first: {errors[0]}")
    warm = max(1, n // 20)
    ls = np.array(lat[warm:])
    third = max(1, len(ls) // 3)
    return {"precision": prec, "offered_rps": rate, "requests": n, "achieved_rps": n / (t1 - t0),
            "p50_ms": float(np.percentile(ls, 50)), "p99_ms": float(np.percentile(ls, 99)),
            "mean_ms": float(ls.mean()),
            # queue trend: median latency of the first and last third of the arrivals
            "p50_first_third_ms": float(np.median(ls[:third])), "p50_last_third_ms": float(np.median(ls[-third:]))}


def _plain_run(S, data, rate, seed):
    """The plain single-instance FP64 path as a server: requests arrive as in
    _served_run and are decomposed and reconstructed one at a time, in
    arrival order, with the synchronous calls; latency = completion minus
    arrival."""
    import numpy as np
    ctx = S.Context(0)
    n = len(data)
    rng = np.random.default_rng(seed)
    arrive = np.cumsum(rng.exponential(1.0 / rate, n))
    lat = []
    t0 = time.perf_counter()
    for i, q in enumerate(data):
        dt = t0 + arrive[i] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        _run_sync(ctx, q, "fp64")
        lat.append(1e3 * (time.perf_counter() - t0 - arrive[i]))
    t1 = time.perf_counter()
    ctx.close()
    warm = max(1, n // 20)
    ls = np.array(lat[warm:])
    return {"precision": "fp64 plain", "offered_rps": rate, "requests": n, "achieved_rps": n / (t1 - t0),
            "p50_ms": float(np.percentile(ls, 50)), "p99_ms": float(np.percentile(ls, 99)),
            "mean_ms": float(ls.mean())}


def _keeps_up(run):
    """A Poisson run the server sustained: it completed at the offered rate and
    the latency did not grow over the run (no queue build-up)."""
    return (run["achieved_rps"] >= 0.95 * run["offered_rps"]
            and run["p50_last_third_ms"] <= 2.0 * max(run["p50_first_third_ms"], 1.0))


def serve_bench(S, W, n_req):
    """Mixed serving workload (60% 1D, 25% MSSA, 15% 2D, r ~ U{5..40},
    groups {1..min(r,4)}): capacity of the plain single-instance FP64 path
    (closed loop), then Poisson arrivals at 0.8 x that capacity through the
    plain path (one request at a time) and the serving engine in FP32 and
    FP64.  The served FP32 capacity is the highest
    Poisson rate it sustains (a ladder of rates below the closed-loop
    throughput, where all requests wait at once and form the largest
    batches); the last run is at 0.8 x that sustained capacity."""
    mix = W.serving_mix(n_req, seed=5)
    data = [W.materialize(d) for d in mix]
    ctx = S.Context(0)
    ncap = min(len(data), 60)
    for q in data[:3]:
        _run_sync(ctx, q, "fp64")
    t0 = time.perf_counter()
    for q in data[:ncap]:
        _run_sync(ctx, q, "fp64")
    cap64 = ncap / (time.perf_counter() - t0)
    ctx.close()
    out = {"workload": f"serving mix, {n_req} requests (60% 1D N~U(500,20000), 25% MSSA s~U(4,32), "
                       f"15% 2D S~U(64,512)), r~U(5,40)",
           "plain_fp64_capacity_rps": cap64, "runs": []}
    # the same arrivals (seed 11) through the plain path and the serving engine
    out["runs"].append(_plain_run(S, data, 0.8 * cap64, seed=11))
    for prec in ("fp32", "fp64"):
        out["runs"].append(_served_run(S, data, prec, 0.8 * cap64, seed=11))
    closed = _served_run(S, data, "fp32", None, seed=12)
    out["served_fp32_closed_loop_rps"] = closed["achieved_rps"]
    sustained, ladder = None, []
    for f in (0.8, 0.65, 0.5, 0.4, 0.3, 0.2):
        rate = f * closed["achieved_rps"]
        if rate <= cap64:
            break
        run = _served_run(S, data, "fp32", rate, seed=14)
        ladder.append({"offered_rps": rate, "achieved_rps": run["achieved_rps"], "p50_ms": run["p50_ms"],
                       "p99_ms": run["p99_ms"], "kept_up": _keeps_up(run)})
        if _keeps_up(run):
            sustained = rate
            break
    out["served_fp32_ladder"] = ladder
    out["served_fp32_capacity_rps"] = sustained
    if sustained:
        out["runs"].append(_served_run(S, data, "fp32", 0.8 * sustained, seed=13))
    return out


# kernel classes timed in the timed region -> kernel names
KERNELS = {"col": "k_colr", "row_mid": "k_rowr_mid"}
PROFILE_EVERY = 7


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel sources have changed since the counters
    were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_image512_batch64_fp32_traffic.md")
    if not os.path.exists(path):
        return None, None
    vals = {}
    for line in open(path):
        line = line.strip()
        for key in ("traffic-bytes-per-launch:", "source-sha256:", "kernel-instance:"):
            if line.startswith(key):
                vals[key] = line[len(key):].strip()
    h = hashlib.sha256()
    for f in ("common.hpp", "device.hpp", "fft.hpp", "regfft.hpp", "kernels.hip"):
        with open(os.path.join(ROOT, "paper_1309_5050_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if vals.get("source-sha256:") != h.hexdigest() or "traffic-bytes-per-launch:" not in vals:
        return None, vals.get("kernel-instance:")
    return float(vals["traffic-bytes-per-launch:"]), vals.get("kernel-instance:")


def cpu_baseline(x, lw):
    """The oracle's explicit S = X X^T formation on a slice of rows of one
    decomposition of the same workload, scaled to a whole decomposition.
    The Jacobi eigen-decomposition of S and the averaging are left out, so
    the true oracle rate is lower than the figure reported."""
    import numpy as np

    import oracle
    t0 = time.perf_counter()
    sh = oracle.shapes(x, window=(lw, lw))
    X = oracle.trajectory(x, sh)
    t_traj = time.perf_counter() - t0
    rows = 48
    t1 = time.perf_counter()
    oracle.gram_rows(X, 0, rows)
    t_slice = time.perf_counter() - t1
    L = X.shape[0]
    full = t_traj + t_slice * (L * L / 2.0) / (rows * L)
    return {"value": 1.0 / full, "unit": "decomps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"explicit trajectory matrix ({L}x{X.shape[1]}) + S=XX^T rows 0..{rows - 1} of {L}, "
                      f"scaled to the full S; Jacobi eigen step and averaging not included (upper bound)",
            "seconds_measured": t_traj + t_slice}


if __name__ == "__main__":
    main()
