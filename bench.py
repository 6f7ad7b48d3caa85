"""Benchmark: batched Shaped 2D-SSA decompositions + reconstructions per second.

Headline workload: the 2D-SSA image workload -- 512x512 images, each a sum of
three planar cosines (periods 8..64 px, random directions) plus N(0, 0.2^2)
noise, window 64x64, r = 30 eigentriples, reconstruction of the groups
{1,2}, {3,4}, {5,6} (0-based {0,1}, {2,3}, {4,5}).  A step decomposes and
reconstructs one batch of B images already resident in device memory.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--batch 768] [--precision fp32]

Prints one JSON line.  Besides the headline rate it reports:

* ``roofline``: the whole FFT product (X v and X^T u) against the HBM peak,
  with the algorithmic bytes per product B_mv = b (K + L) + 2 b M_A (M_B/2 + 1)
  (vector in, vector out, spectrum read once; b = 4 for FP32 products, 8 for
  FP64) times the products of the timed batches, over the summed HIP-event
  time of the product kernels in the timed region (one launch in seven of
  each class timed, scaled by the class's launch count).  ``roofline_kernels``
  splits it by kernel class, each with the part of B_mv it moves.
* the same batched measurement in FP64 and for the 1D, MSSA and shaped
  workloads, the plain single-instance FP64 path, the paper's own timing
  experiments on a Mars-like stand-in, and the CPU oracle timed on the host.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
PROFILE_EVERY = 7
# kernel classes of the FFT product (the library's timing classes) and the
# kernels behind them on the register (power-of-two) path
GRID_CLASSES = ["row_in", "col", "row_mid", "row_out"]
ROWFAM_CLASSES = ["row_in", "rowfam_mid", "rowfam_out"]
KERNEL_OF = {"row_in": "k_rowr_in", "col": "k_colr", "row_mid": "k_rowr_mid", "row_out": "k_rowr_out",
             "rowfam_mid": "k_row_mid", "rowfam_out": "k_row_out"}
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "fft_product_image512_batch768_fp32_traffic.md")
# the paper's decomposition timings (R, Rssa 0.10 with FFTW; hardware not
# stated), elapsed seconds, for the three settings on its 258 x 275 image
PAPER_SECONDS = {"eigen_25x25": 3.843, "lanczos_25x25": 0.519, "lanczos_160x80_r50": 0.587,
                 "shaped_circle15_mask": 0.684}


def _prec_bytes(prec):
    return 8 if prec == "fp64" else 4


def bmv_of(d, prec):
    """Algorithmic bytes of one product of decomposition d."""
    st = d.stats
    b = _prec_bytes(prec)
    return b * (d.K + d.L) + 2 * b * st["fft_rows"] * (st["fft_cols"] // 2 + 1)


def class_bytes(ds, prec, rowfam):
    """Part of the timed products' algorithmic bytes each kernel class moves.
    Per step (two products): the input pass reads the short-side vector, the
    column passes read the spectrum once per product, the middle pass writes
    the long-side result of the first product and reads the long-side input
    of the second, the output pass writes the short-side result."""
    b = _prec_bytes(prec)
    out = {}
    for d in ds:
        st = d.stats
        steps = st["steps"]
        nshort, nlong = (d.L, d.K) if st["side"] == 0 else (d.K, d.L)
        xh = 2 * b * st["fft_rows"] * (st["fft_cols"] // 2 + 1)
        if rowfam:
            parts = {"row_in": b * nshort, "rowfam_mid": 2 * b * nlong + xh, "rowfam_out": b * nshort + xh}
        else:
            parts = {"row_in": b * nshort, "col": 2 * xh, "row_mid": 2 * b * nlong, "row_out": b * nshort}
        for k, v in parts.items():
            out[k] = out.get(k, 0.0) + steps * v
    return out


def measured_traffic(batch):
    """Counter bytes per dispatch of each product kernel from the committed
    rocprofv3 summary, or None when the kernel sources have changed since
    the counters were taken or the summary is of another batch size."""
    import hashlib
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    per, sha, tb = {}, None, None
    for line in open(TRAFFIC_SUMMARY):
        f = line.split()
        if len(f) >= 2 and f[0] == "source-sha256:":
            sha = f[1]
        if len(f) == 2 and f[0] == "batch:":
            tb = int(f[1])
        if len(f) == 4 and f[0] == "traffic:":
            per[f[1]] = (float(f[2]), float(f[3]))   # class -> (bytes per dispatch, dispatches counted)
    h = hashlib.sha256()
    for f in ("common.hpp", "device.hpp", "fft.hpp", "regfft.hpp", "kernels.hip"):
        with open(os.path.join(ROOT, "paper_1309_5050_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return per if sha == h.hexdigest() and per and tb == batch else None


def product_roofline(prof, ds, prec, rowfam, nbatch, traffic=None):
    """Whole-product roofline and per-class entries from a profile record of
    nbatch timed batches, all like the batch ds (the same inputs each time,
    so the same steps)."""
    classes = ROWFAM_CLASSES if rowfam else GRID_CLASSES
    cb = {k: nbatch * v for k, v in class_bytes(ds, prec, rowfam).items()}
    products = nbatch * 2 * sum(d.stats["steps"] for d in ds)
    bmv_total = nbatch * sum(2 * d.stats["steps"] * bmv_of(d, prec) for d in ds)
    kern, t_total = {}, 0.0
    for c in classes:
        p = prof[c]
        if p["launches"] == 0:
            continue
        per_launch = p["ms"] / p["launches"]
        ms = per_launch * p["all_launches"]
        t_total += ms
        gbs = cb[c] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        kern[c] = {"kernel": KERNEL_OF[c], "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": gbs / HBM_PEAK_GBS, "ms_per_launch": per_launch, "launches": p["all_launches"],
                   "launches_timed": p["launches"], "ms_total": ms,
                   "bytes_per_launch": cb[c] / max(p["all_launches"], 1)}
    ach = bmv_total / (t_total * 1e-3) / 1e9 if t_total > 0 else 0.0
    tr = None
    if traffic:
        counted = sum(traffic[c][0] * kern[c]["launches"] for c in kern if c in traffic)
        if all(c in traffic for c in kern):
            tr = counted / products
    bmv_mean = bmv_total / max(products, 1)
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": tr,
            "kernel": "FFT product: " + " + ".join(KERNEL_OF[c] for c in classes),
            "unit_of_work": "one product X v or X^T u", "bytes_per_product": bmv_mean, "products": products,
            "ms_total": t_total, "us_per_product": 1e3 * t_total / max(products, 1),
            "traffic_over_bmv": (tr / bmv_mean) if tr else None, "timed_every": PROFILE_EVERY}
    return roof, kern


def run_batched(S, ctx, torch, xs, window, r, groups, prec, steps, warmup, masks=None, extra_classes=()):
    """Time `steps` batches (decompose + reconstruct, inputs on the device)
    after `warmup` untimed ones; returns (decomps/s, ms per step, the last
    batch's handles, the profile record)."""
    dev = xs[0].device
    outs = [torch.empty((len(groups),) + tuple(x.shape), dtype=torch.float64, device=dev) for x in xs]

    def step():
        ds = ctx.decompose_batch_dev(xs, window, r, precision=prec, masks=masks)
        bad = [d for d in ds if isinstance(d, Exception)]
        if bad:
            raise bad[0]
        S.Context.reconstruct_batch_dev(ds, groups, outs)
        return ds

    for _ in range(warmup):
        ds = step()
        del ds
    torch.cuda.synchronize()
    rowfam = None
    kinds = GRID_CLASSES + ROWFAM_CLASSES[1:] + list(extra_classes)
    ctx.profile(",".join(kinds), every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(steps):
        last = None          # a step's results are released before the next step
        last = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read(kinds)
    ctx.profile(None)
    rowfam = prof["col"]["all_launches"] == 0
    dt = t1 - t0
    return len(xs) * steps / dt, 1e3 * dt / steps, last, prof, rowfam


def note(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def config_line(S, W, ctx, torch, which, prec, steps, warmup, batch=None):
    """Batched rate and product roofline of one of the other workloads
    (batch: instances per batch call, default the workload's own)."""
    import numpy as np
    note(f"workload {which} ({prec})")
    dev = torch.device("cuda:0")
    if which == 1:
        B, groups = batch or 1024, [[0, 1], [2, 3], [4]]
        ws = [W.series_1d(seed=1 + i) for i in range(B)]
        # a series as a one-row array with a one-row window (the same
        # trajectory matrix as the column orientation)
        xs = [torch.tensor(w["x"][None, :], device=dev) for w in ws]
        masks, window, r = None, (1, ws[0]["window"]), ws[0]["r"]
        name = "1D SSA N=1000, L=500, r=10, groups {1,2},{3,4},{5}"
    elif which == 3:
        B, groups = batch or 1024, [[0, 1], [2, 3]]
        ws = [W.mssa_series(seed=3 + i) for i in range(B)]
        xs = []
        for w in ws:
            nmax = max(len(s) for s in w["x"])
            arr = np.full((len(w["x"]), nmax), np.nan)      # one series per row, NaN after each end
            for p, s in enumerate(w["x"]):
                arr[p, :len(s)] = s
            xs.append(torch.tensor(arr, device=dev))
        masks, window, r = None, (1, ws[0]["window"]), ws[0]["r"]
        name = "MSSA 50 series N~U(1000,3000), L=500, r=20, groups {1,2},{3,4}"
    else:
        B, groups = batch or 256, [[0, 1, 2, 3]]
        ws = [W.shaped_disc(seed=4 + i) for i in range(B)]
        xs = [torch.tensor(w["x"], device=dev) for w in ws]
        masks = [torch.tensor(w["mask"], device=dev) for w in ws]
        window, r = ws[0]["window"], ws[0]["r"]
        name = "shaped 1024x1024 disc r=480 with 10% NaN holes, 32x32 window, r=50, group {1..4}"
    rate, ms, last, prof, rowfam = run_batched(S, ctx, torch, xs, window, r, groups, prec, steps, warmup,
                                               masks=masks)
    roof, kern = product_roofline(prof, last, prec, rowfam, steps)
    return {"workload": name, "batch": B, "precision": prec, "decomps_per_s": rate, "ms_per_step": ms,
            "roofline": roof, "roofline_kernels": kern,
            "lanczos_steps_mean": float(np.mean([d.stats["steps"] for d in last]))}


def continuous_line(S, W, ctx, torch, xs0, window, r, groups):
    """Twice the headline batch of images (the headline's images, each
    twice): two lockstep batch calls of one batch each against one call of
    all of them through as many slots as a batch holds (continuous batching:
    images start as others finish, so the calls' convergence tails overlap).
    Decompositions + reconstructions per second, inputs on the device."""
    dev = xs0[0].device
    nb = len(xs0)
    xs = list(xs0) + [x.clone() for x in xs0]
    n = len(xs)
    outs = [torch.empty((len(groups),) + tuple(x.shape), dtype=torch.float64, device=dev) for x in xs]

    def run(parts, slots):
        ctx.set_slots(slots)
        for p in parts:
            ds = ctx.decompose_batch_dev([xs[i] for i in p], window, r, precision="fp32")
            S.Context.reconstruct_batch_dev(ds, groups, [outs[i] for i in p])
            del ds
        torch.cuda.synchronize()

    lock = [list(range(k, k + nb)) for k in range(0, n, nb)]
    one = [list(range(n))]
    run(lock[:1], 0)                                  # warm-ups (the memory pool grows to each call's size)
    run(one, nb)
    t0 = time.perf_counter()
    run(lock, 0)
    t1 = time.perf_counter()
    run(one, nb)
    t2 = time.perf_counter()
    ctx.set_slots(0)
    return {"workload": f"{n} images 512x512 (the headline's {nb}, each twice), 64x64 window, r=30, fp32",
            "lockstep_decomps_per_s": n / (t1 - t0), "lockstep_calls": len(lock), "lockstep_batch": nb,
            "one_call_decomps_per_s": n / (t2 - t1), "slots": nb}


def paper_context(S, W, torch):
    """The paper's decomposition timings re-run on a synthetic Mars-like
    stand-in (258 x 275, bright disc on a zero = NA background, planar sines
    of periods near 5 and 10 px), single decompositions in FP64 from host
    inputs, r = 50 (the package's default number of eigentriples)."""
    import numpy as np
    w = W.mars_like()
    x, mask = w["x"], w["mask"]
    full = np.nan_to_num(x)          # the plain 2D-SSA runs decompose the whole array
    ctx = S.Context(0)
    out = {"workload": "Mars-like 258x275 stand-in, FP64, r=50, single decomposition from host memory",
           "paper_seconds_hardware": "not stated (R, Rssa 0.10, FFTW)", "runs": {}}

    def timed(fn, reps=3):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            d = fn()
            _ = d.sigma
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            d.free()
            best = t if best is None else min(best, t)
        return best

    cases = {
        "lanczos_25x25": lambda: ctx.decompose(full, (25, 25), 50),
        "lanczos_160x80_r50": lambda: ctx.decompose(full, (160, 80), 50),
        "shaped_circle15_mask": lambda: ctx.decompose(x, w["window"], 50, mask=mask, wmask=w["wmask"]),
        "eigen_25x25": lambda: ctx.decompose(full, (25, 25), 50, method="eigen"),
    }
    for k, fn in cases.items():
        try:
            t = timed(fn)
            out["runs"][k] = {"seconds": t, "paper_seconds": PAPER_SECONDS[k], "paper_over_ours": PAPER_SECONDS[k] / t}
        except S.SsaError as e:
            out["runs"][k] = {"seconds": None, "paper_seconds": PAPER_SECONDS[k], "error": str(e)}
    ctx.close()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(W):
    """The CPU oracle (explicit trajectory matrix, one-sided Jacobi SVD,
    averaging by explicit summation) timed on the host: complete
    decompositions + reconstructions of the reduced 2D workload (128x128
    image, 16x16 window, r = 30, groups {1,2},{3,4},{5,6}) and of the 1D
    workload, with every host thread and with one."""
    import oracle
    from threadpoolctl import threadpool_limits

    def one(w, groups):
        t0 = time.perf_counter()
        sh, s, U, V = oracle.decompose(w["x"], window=w["window"])
        for g in groups:
            oracle.reconstruct(sh, s, U, V, g)
        return time.perf_counter() - t0

    w2 = W.config(2, "small")
    w1 = W.config(1)
    g2, g1 = [[0, 1], [2, 3], [4, 5]], [[0, 1], [2, 3], [4]]
    allc = oracle.num_threads()
    t2 = one(w2, g2)
    t1 = one(w1, g1)
    oracle.set_threads(1)
    with threadpool_limits(limits=1):
        t2s = one(w2, g2)
        t1s = one(w1, g1)
    oracle.set_threads(allc)
    return {"value": 1.0 / t2, "unit": "decomps/s", "cores": allc, "kind": "oracle",
            "sample": "complete oracle decomposition + reconstruction of the reduced 2D workload "
                      "(128x128 image, 16x16 window: X is 256 x 12769; r=30, 3 groups), all host threads",
            "cpu_model": cpu_model(), "single_thread_decomps_per_s": 1.0 / t2s,
            "seconds": {"reduced_2d_all_threads": t2, "reduced_2d_one_thread": t2s,
                        "series_1000_all_threads": t1, "series_1000_one_thread": t1s},
            "recorded_full_512x512": {"seconds": 660.0, "threads": 8, "route": "S = X X^T + Jacobi eigenpairs",
                                      "note": "one run of tests/golden/make_golden.py 2 on the 8-core "
                                              "build host (Xeon, 2.70 GHz), not re-timed here"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=768)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "fp32_basis32"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--no-single", action="store_true", help="skip the single-instance FP64 comparator")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the w-correlation, forecast, continuation and eigen-method timings")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the FP64, 1D, MSSA, shaped and paper-context lines")
    ap.add_argument("--serve", type=int, default=300, metavar="N",
                    help="requests of the mixed serving workload for the latency runs through the "
                         "batch calls (0: skip)")
    ap.add_argument("--serve-coop", type=int, default=300, metavar="N",
                    help="requests of the serving mix through the cooperative server (0: skip)")
    ap.add_argument("--serve-engine", type=int, default=0, metavar="N",
                    help="requests for the library's asynchronous serving engine (ssa_submit); off by "
                         "default: its worker-thread path is not run on the GPU until a fault seen on an "
                         "earlier build is explained")
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

    note("headline batches")
    value, ms_step, last, prof, rowfam = run_batched(S, ctx, torch, xs, (lw, lw), r, groups, args.precision,
                                                     args.steps, args.warmup, extra_classes=("lz_ritz", "lz_svd"))
    roof, kern = product_roofline(prof, last, args.precision, rowfam, args.steps,
                                  measured_traffic(B) if args.precision == "fp32" else None)
    stats = last[0].stats
    st_all = sorted(d.stats["steps"] for d in last)
    steps_dist = [st_all[0], st_all[len(st_all) // 2], st_all[-1]]
    # Jacobi sweeps per projected-matrix SVD (one SVD per restart cycle)
    sweeps_per_svd = (sum(d.stats["svd_sweeps"] for d in last) /
                      max(1, sum(d.stats["restarts"] + 1 for d in last)))
    # measured orthonormality of the results (outside the timed region): the
    # worst over the first 16 results of the last batch
    orth = [d.orthogonality() for d in last[:16]]
    orth = {"max_UtU_minus_I": max(o[0] for o in orth), "max_VtV_minus_I": max(o[1] for o in orth),
            "results": len(orth)}
    # the matrix-core kernel (FP64 Ritz rotation): its timing class counts
    # floating-point operations
    pr = prof["lz_ritz"]
    mfma = None
    if pr["launches"] > 0 and pr["ms"] > 0:
        tf = pr["bytes"] / (pr["ms"] * 1e-3) / 1e12
        mfma = {"kernel": "k_lz_ritz", "dtype": "f64", "achieved": tf, "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": tf / FP64_MFMA_PEAK_TFLOPS, "launches": pr["launches"],
                "ms_per_launch": pr["ms"] / pr["launches"], "flop_per_launch": pr["bytes"] / pr["launches"]}

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

        # continuation: one decomposition of the workload extended by r/5
        # triplets, against decomposing it afresh with that many
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
        # a series longer than one transform row (decomposed in segments):
        # 200,000 values, L = 1000, r = 10, FP64, with reconstruction
        xlong = W.series_1d(n=200000, L=1000, r=10)["x"]
        d0 = ctx.decompose(xlong[:16384], 1000, 2)     # the segments' row length: kernels loaded
        d0.free()
        torch.cuda.synchronize()
        tl0 = time.perf_counter()
        dlong = ctx.decompose(xlong, 1000, 10)
        _ = dlong.sigma
        tl1 = time.perf_counter()
        reclong = dlong.reconstruct([[0, 1], [2, 3]])
        tl2 = time.perf_counter()
        eigen["long_series"] = {"workload": "1D series N=200000, L=1000, r=10, fp64 (in segments of 16384 values)",
                                "decompose_ms": 1e3 * (tl1 - tl0), "reconstruct_ms": 1e3 * (tl2 - tl1),
                                "steps": dlong.stats["steps"], "finite": bool(np.isfinite(reclong).all())}
        dlong.free()
        return wcor, rforecast, extend, eigen

    wcor = rforecast = extend = eigen = None
    if not args.no_extras:
        note("extras")
        wcor, rforecast, extend, eigen = run_extras()
    del last
    # the lines below run in contexts of their own, each closed after it, so
    # that one line's memory pool is returned before the next grows its own
    # (the headline's pool holds a batch of 768 images' blocks)
    def fresh():
        return S.Context(0, stream=stream.cuda_stream)

    def done(c):
        c.close()
        torch.cuda.empty_cache()

    done(ctx)
    ctx = fresh()

    # the same workload in FP64 (the paper's arithmetic), the other workloads,
    # the reduced 2D workload the CPU oracle is timed on, and the paper's own
    # timing experiments
    configs = paper = None
    if not args.no_configs:
        configs = {}

        def guarded(name, fn, len_tune=False):
            """One line in a context of its own.  A library error (say, an
            allocation refused) is reported in the line's place instead of
            ending the run."""
            if len_tune:
                os.environ["SHSSA_LEN_TUNE"] = "1"
            c = fresh()
            if len_tune:
                del os.environ["SHSSA_LEN_TUNE"]
            try:
                configs[name] = fn(c)
            except S.SsaError as e:
                note(f"{name}: {e}")
                configs[name] = {"error": str(e)}
            finally:
                done(c)

        def fp64_line(c):
            n64 = max(2, args.steps // 2)
            rate64, ms64, last64, prof64, rf64 = run_batched(S, c, torch, xs, (lw, lw), r, groups, "fp64", n64, 1)
            roof64, kern64 = product_roofline(prof64, last64, "fp64", rf64, n64)
            return {"workload": "2D-SSA 512x512 image, 64x64 window, r=30 (as the headline)",
                    "batch": B, "precision": "fp64", "decomps_per_s": rate64, "ms_per_step": ms64,
                    "roofline": roof64, "roofline_kernels": kern64}

        def reduced_line(c):
            w2 = W.config(2, "small")
            xr = [torch.tensor(W.image_2d(n=128, lw=16, r=30, seed=2000 + i)["x"], device=dev) for i in range(64)]
            rr, msr, _, _, _ = run_batched(S, c, torch, xr, w2["window"], 30, groups, "fp64", 3, 1)
            return {"workload": "reduced 2D-SSA 128x128 image, 16x16 window, r=30 "
                                "(the workload the CPU oracle is timed on)",
                    "batch": 64, "precision": "fp64", "decomps_per_s": rr, "ms_per_step": msr}

        note("headline workload in fp64")
        guarded("image512_fp64", fp64_line)
        guarded("series_1000_fp64", lambda c: config_line(S, W, c, torch, 1, "fp64", 3, 1))
        # the same with the length tuner on (half-length 500 or 512, timed on
        # the first request; the warm-up batch carries the tuning)
        guarded("series_1000_fp64_length_tuned", lambda c: config_line(S, W, c, torch, 1, "fp64", 3, 1),
                len_tune=True)
        guarded("mssa_50_fp32", lambda c: config_line(S, W, c, torch, 3, "fp32", 3, 1))
        guarded("shaped_1024_fp32", lambda c: config_line(S, W, c, torch, 4, "fp32", 2, 1))
        guarded("image128_fp64", reduced_line)
        note("continuous batching")
        try:
            configs["continuous_image512_fp32"] = continuous_line(S, W, ctx, torch, xs, (lw, lw), r, groups)
        except S.SsaError as e:
            note(f"continuous batching: {e}")
            configs["continuous_image512_fp32"] = {"error": str(e)}
        note("paper context")
        paper = paper_context(S, W, torch)

    # plain single-instance FP64 path (same kernels, batch of one)
    single = None
    if not args.no_single:
        outs1 = [torch.empty((len(groups), n, n), dtype=torch.float64, device=dev) for _ in range(2)]
        reps = 2
        # untimed: the context's first FP64 call carries the column tuning
        d = ctx.decompose_batch_dev(xs[:1], (lw, lw), r, precision="fp64")[0]
        S.Context.reconstruct_batch_dev([d], groups, outs1[:1])
        del d
        torch.cuda.synchronize()
        lat = []
        for i in range(reps):
            ta = time.perf_counter()
            d = ctx.decompose_batch_dev(xs[i:i + 1], (lw, lw), r, precision="fp64")[0]
            S.Context.reconstruct_batch_dev([d], groups, outs1[i:i + 1])
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - ta)
        single = {"decomps_per_s": reps / sum(lat), "latency_ms": 1e3 * float(np.median(lat))}

    serving = None
    if args.serve > 0:
        note("serving loop")
        serving = serve_batched(S, W, args.serve)
    if args.serve_coop > 0:
        note("cooperative server")
        cap = serving.get("plain_fp64_capacity_rps") if serving else None
        serving = dict(serving or {}, coop=serve_bench(S, W, args.serve_coop, cap64=cap, plain=cap is None))
    if args.serve_engine > 0:
        os.environ["SHSSA_SERVE_ENGINE"] = "1"   # the library keeps its serving threads off otherwise
        serving = dict(serving or {}, engine=serve_bench(S, W, args.serve_engine))

    cpu = None
    if not args.no_cpu:
        note("cpu oracle")
        cpu = cpu_baseline(W)
        if configs and "decomps_per_s" in configs.get("image128_fp64", {}):
            cpu["gpu_over_oracle_same_workload"] = configs["image128_fp64"]["decomps_per_s"] / cpu["value"]

    line = {
        "metric": "SSA decomps/s (decompose r=30 + reconstruct 3 groups), 512x512 image, 64x64 window",
        "value": value,
        "unit": "decomps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "2D-SSA 512x512 image, 64x64 window, r=30, groups {1,2},{3,4},{5,6}",
                   "batch": B, "precision": args.precision + (" products, fp64 Lanczos" if
                                                             args.precision != "fp64" else ""),
                   "parallelism": "batched on 1 GPU"},
        "roofline": roof,
        "roofline_kernels": kern,
        "mfma": mfma,
        "lanczos": {"steps": stats["steps"], "restarts": stats["restarts"], "basis": stats["basis"],
                    "max_resid_over_sigma1": stats["max_resid"],
                    "steps_min_median_max": steps_dist,
                    "svd_launches_per_batch": prof["lz_svd"]["all_launches"] / max(args.steps, 1),
                    "svd_ms_per_launch": (prof["lz_svd"]["ms"] / prof["lz_svd"]["launches"]
                                          if prof["lz_svd"]["launches"] else None),
                    "svd_sweeps_per_svd": sweeps_per_svd, "orthogonality": orth},
        "host_ms_per_batch": {"setup": B * stats["ms_setup"], "lanczos": B * stats["ms_lanczos"],
                              "finish": B * stats["ms_finish"]},
        "fp64_single_instance": single,
        "speedup_vs_fp64_single": (value / single["decomps_per_s"]) if single else None,
        "configs": configs,
        "paper_context": paper,
        "wcor": wcor,
        "rforecast": rforecast,
        "extend": extend,
        "eigen": eigen,
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


def _as_request(q):
    """A serving-mix request as a batch-call request: series as they are,
    MSSA series side by side in one array (NaN after each series' end) with
    an L x 1 window, the packing of ssa_decompose_multi."""
    import numpy as np
    if q["kind"] == "mssa":
        nmax = max(len(x) for x in q["x"])
        arr = np.full((nmax, len(q["x"])), np.nan)
        for p, x in enumerate(q["x"]):
            arr[:len(x), p] = x
        return {"x": arr, "window": (q["window"], 1), "r": q["r"]}
    return {"x": q["x"], "window": q["window"], "r": q["r"], "mask": q.get("mask"), "wmask": q.get("wmask")}


def _size_class(q):
    """Request kind and transform size class (row kernel class of the series
    length, or the image side's power of two): requests that would share
    the library's kernel launches."""
    if q["kind"] == "2d":
        n = q["x"].shape[0]
        return ("2d", (n - 1).bit_length(), q["x"].shape[0] // max(q["window"][0], 1))
    n = max(len(x) for x in q["x"]) if q["kind"] == "mssa" else len(q["x"])
    half = (n + 1) // 2
    return (q["kind"], 0 if half <= 512 else 1 if half <= 2048 else 2)


def _batched_server_run(S, data, reqs, prec, rate, seed, max_batch=64):
    """A server loop over the batch calls: requests arrive as a Poisson
    process; whenever the GPU is free, the oldest waiting request and the
    arrived requests of its size class that follow it (up to max_batch) go
    into one batch call (they share launches; at most 64 of a class advance
    together, the others take the slots of finished ones), then each result
    is reconstructed.
    Latency = the time its reconstruction is on the host minus its arrival;
    the first 5% of requests are warm-up and left out."""
    import numpy as np
    ctx = S.Context(0)
    ctx.set_slots(64)
    n = len(data)
    rng = np.random.default_rng(seed)
    arrive = np.cumsum(rng.exponential(1.0 / rate, n))
    lat = np.zeros(n)
    sizes = []
    t0 = time.perf_counter()
    i = 0
    while i < n:
        now = time.perf_counter() - t0
        if arrive[i] > now:
            time.sleep(arrive[i] - now)
            now = time.perf_counter() - t0
        # the arrived requests of the first one's size class (requests of
        # one class share every launch; a call returns when all its requests
        # are done, so other classes go into calls of their own)
        j = i + 1
        while j < n and arrive[j] <= now and j - i < max_batch and _size_class(data[j]) == _size_class(data[i]):
            j += 1
        ds = ctx.decompose_batch(reqs[i:j], precision=prec)
        for k, d in zip(range(i, j), ds):
            if isinstance(d, Exception):
                raise RuntimeError(f"request {k}: {d}")
            d.reconstruct(data[k]["groups"])      # returns when the request's results are on the host
            d.free()
            lat[k] = 1e3 * (time.perf_counter() - t0 - arrive[k])
        sizes.append(j - i)
        i = j
    t1 = time.perf_counter()
    ctx.close()
    ls = lat[max(1, n // 20):]
    return {"precision": prec, "offered_rps": rate, "requests": n, "achieved_rps": n / (t1 - t0),
            "p50_ms": float(np.percentile(ls, 50)), "p99_ms": float(np.percentile(ls, 99)),
            "mean_ms": float(ls.mean()), "batches": len(sizes), "mean_batch": float(np.mean(sizes))}


def serve_batched(S, W, n_req):
    """Mixed serving workload (60% 1D N ~ U{500..20000}, L = N/2; 25% MSSA of
    4..32 series; 15% 2D images of side 64..512 with an (S/8)^2 window;
    r ~ U{5..40}; groups {1..min(r,4)}), Poisson arrivals at 0.8 x the
    closed-loop capacity of the plain single-instance FP64 path: that path
    (one request at a time, synchronous calls) against the batched server
    loop in FP32 and FP64 at the same arrivals, then the batched FP32 loop
    at higher rates (1.25, 1.5, 2, 3 x the plain capacity, up to the first
    it does not sustain)."""
    mix = W.serving_mix(n_req, seed=5)
    data = [W.materialize(d) for d in mix]
    reqs = [_as_request(q) for q in data]
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
                       f"15% 2D S~U(64,512)), r~U(5,40), Poisson arrivals",
           "server": "batch calls of the requests that have arrived (64 slots per kernel class)",
           "plain_fp64_capacity_rps": cap64, "runs": []}
    out["runs"].append(_plain_run(S, data, 0.8 * cap64, seed=11))
    for prec in ("fp32", "fp64"):
        out["runs"].append(_batched_server_run(S, data, reqs, prec, 0.8 * cap64, seed=11))
    ladder = []
    for f in (1.25, 1.5, 2.0, 3.0):
        run = _batched_server_run(S, data, reqs, "fp32", f * cap64, seed=14)
        run["kept_up"] = run["achieved_rps"] >= 0.95 * run["offered_rps"]
        ladder.append(run)
        if not run["kept_up"]:
            break
    out["fp32_ladder"] = ladder
    return out


def _keeps_up(run):
    """A Poisson run the server sustained: it completed at the offered rate and
    the latency did not grow over the run (no queue build-up)."""
    return (run["achieved_rps"] >= 0.95 * run["offered_rps"]
            and run["p50_last_third_ms"] <= 2.0 * max(run["p50_first_third_ms"], 1.0))


def serve_bench(S, W, n_req, cap64=None, plain=True):
    """Mixed serving workload (60% 1D, 25% MSSA, 15% 2D, r ~ U{5..40},
    groups {1..min(r,4)}) through ssa_submit / ssa_wait / ssa_take (the
    cooperative server, or the worker threads with SHSSA_SERVE_ENGINE):
    capacity of the plain single-instance FP64 path (closed loop; cap64 when
    already measured), then Poisson arrivals at 0.8 x that capacity through
    the plain path (one request at a time; plain = False: measured
    elsewhere at the same arrivals) and the server in FP32 and FP64.  The
    served FP32 capacity is the highest Poisson rate it sustains (a ladder of
    rates below the closed-loop throughput, where all requests wait at once
    and form the largest batches); the last run is at 0.8 x that sustained
    capacity."""
    mix = W.serving_mix(n_req, seed=5)
    data = [W.materialize(d) for d in mix]
    if cap64 is None:
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
           "server": ("library worker threads" if os.environ.get("SHSSA_SERVE_ENGINE") else
                      "cooperative: the collecting thread's waits run admissions and restart cycles; requests "
                      "join running batches as slots free"),
           "plain_fp64_capacity_rps": cap64, "runs": []}
    # the same arrivals (seed 11) through the plain path and the server
    if plain:
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


if __name__ == "__main__":
    main()
