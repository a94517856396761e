"""Throughput benchmark of the fused block-wise approximate DCT on one MI355X.

Workload (the plain method at scale): 1024 synthetic 2048 x 2048 uint8 images
(2D AR(1) fields, rho ~ U[0.85, 0.98] per image, seeded), resident in HBM.
One step is the whole hot path over the batch for every point of the sweep
T in {T1, T2} x r in {1, 6, 10, 16, 28, 45, 64} with N = 8: 14 fused launches,
each doing level shift, forward 2D transform, zig-zag retention, the
orthogonalising scale, the inverse transform, rounding/clipping and the
per-image error energy, and writing the retained int32 coefficients, the
float32 scaled coefficients, the reconstruction and the error energies, each
followed by the float32 PSNR of every image; and, once per transform (they do
not depend on r), the coefficient moments of every image and its float32
measured coding gain.

Prints one JSON line (see the keys below).  ``--gpus N`` with N > 1 exits:
the build targets one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpixel/s fwd+inv 2D approx DCT (batched vs plain), HBM GB/s vs peak; p99 ms"
HBM_PEAK_GBS = 8000.0
SWEEP_R = (1, 6, 10, 16, 28, 45, 64)
KINDS = (1, 2)
N = 8
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_compress8_c1.json")
KERNEL_SOURCES = ("paper_2207_11638_amd/csrc/kernels_n8.hip",
                  "paper_2207_11638_amd/csrc/tile8.hpp",
                  "paper_2207_11638_amd/csrc/butterflies.hpp",
                  "paper_2207_11638_amd/csrc/adct_internal.hpp")


def algorithmic_bytes(b, h, w, r):
    """Bytes one fused launch must move: pixels in and out, retained int32
    coefficients and their float32 scaled values, one error energy per image."""
    tiles = b * (h // N) * (w // N)
    return b * h * w * 2 + tiles * r * (4 + 4) + b * 8


def kernel_source_digest():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per step from the committed rocprofv3 counter summary, or None
    when the kernel source has changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != kernel_source_digest():
        return None
    return t.get("hbm_bytes_per_launch_avg")


COPY_BYTES = 1 << 30


def _read_pmc(d, counter):
    """{kernel name: [value per dispatch]} from a rocprofv3 --pmc csv run."""
    import csv
    import glob
    out = {}
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def summarize_pmc(fetch_dir, write_dir):
    """Counters are KiB per dispatch; each is scaled by what it reads for a plain
    copy kernel of COPY_BYTES (read COPY_BYTES, write COPY_BYTES)."""
    fetch = _read_pmc(fetch_dir, "FETCH_SIZE")
    write = _read_pmc(write_dir, "WRITE_SIZE")

    def pick(d, pred):
        vals = [v for k, vs in d.items() if pred(k) for v in vs]
        return vals

    is_copy = lambda k: "elementwise" in k and "add" in k.lower() or "CUDAFunctor_add" in k
    is_fused = lambda k: "compress8<" in k
    cf, cw = pick(fetch, is_copy), pick(write, is_copy)
    if not cf or not cw:
        raise SystemExit("calibration copy kernel not found in the counter runs")
    fscale = COPY_BYTES / (cf[0] * 1024.0)
    wscale = COPY_BYTES / (cw[0] * 1024.0)
    per = {}
    for name in set(fetch) | set(write):
        if not is_fused(name):
            continue
        f = fetch.get(name, [0.0])
        w = write.get(name, [0.0])
        fb = sum(f) / len(f) * 1024.0 * fscale
        wb = sum(w) / len(w) * 1024.0 * wscale
        per[name] = {"fetch_bytes": fb, "write_bytes": wb}
    if not per:
        raise SystemExit("no fused kernel dispatches in the counter runs")
    avg = sum(v["fetch_bytes"] + v["write_bytes"] for v in per.values()) / len(per)
    out = {"source_digest": kernel_source_digest(), "copy_bytes": COPY_BYTES,
           "fetch_scale": fscale, "write_scale": wscale,
           "hbm_bytes_per_launch_avg": avg, "kernels": per}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps({"hbm_bytes_per_launch_avg": avg, "fetch_scale": fscale,
                      "write_scale": wscale}))


# ------------------------------------------------------------- host workers
# Host-side work (drawing the synthetic inputs, timing the oracle) runs in
# worker processes only while this process has not touched the GPU, and never
# under a profiler: a process that has initialised the GPU (the profiler's
# preloaded library does so at start-up) must not fork, and a pool torn down
# with terminate() SIGTERMs its workers, which the profiler's chained signal
# handler turns into an abort.  Pools here are therefore created before the
# first GPU call and always shut down with close() + join(), so each worker
# leaves through its normal exit path.  Everywhere else threads are used.
_GPU_TOUCHED = False
# worker processes on the GPU machine: its CPU share for one GPU, whatever the
# host's core count is
MAX_WORKERS = 16


def under_profiler() -> bool:
    """True when a rocprofv3 tool library is loaded into this process."""
    return (any(k.startswith(("ROCPROF", "ROCP_")) for k in os.environ)
            or "rocprof" in os.environ.get("LD_PRELOAD", ""))


def host_workers(requested=None) -> int:
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:   # pragma: no cover
        avail = os.cpu_count() or 1
    n = min(avail, MAX_WORKERS)
    return max(1, min(n, requested) if requested else n)


def gpu_device():
    """cuda:0, remembering that the process now uses the GPU."""
    global _GPU_TOUCHED
    import torch
    _GPU_TOUCHED = True
    return torch.device("cuda:0")


class HostPool:
    """map() over worker processes when that is safe (no GPU use yet, no
    profiler), over threads otherwise; closed with close() + join()."""

    def __init__(self, workers: int):
        self.workers = max(1, workers)
        if self.workers > 1 and not _GPU_TOUCHED and not under_profiler():
            import multiprocessing as mp
            self.kind = "processes"
            self.pool = mp.get_context("fork").Pool(self.workers)
        else:
            from multiprocessing.pool import ThreadPool
            self.kind = "threads"
            self.pool = ThreadPool(self.workers)

    def map(self, fn, items, chunksize=1):
        return self.pool.map(fn, items, chunksize=chunksize)

    def imap(self, fn, items, chunksize=1):
        return self.pool.imap(fn, items, chunksize=chunksize)

    def close(self):
        self.pool.close()
        self.pool.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _c1_image(i_hw):
    import synth
    i, h, w = i_hw
    return synth.ar1_batch_image(i, h, w)[0]


def c1_images(pool, b, h, w):
    """Images 0..b-1 of the 2048^2 AR(1) batch (uint8 [b, h, w])."""
    import numpy as np
    imgs = np.empty((b, h, w), dtype=np.uint8)
    for i, img in enumerate(pool.imap(_c1_image, [(i, h, w) for i in range(b)], chunksize=4)):
        imgs[i] = img
    return imgs


# ------------------------------------------------------------------ CPU leg
def _oracle_task(args):
    """One oracle task over one image: a fused pass (r > 0) or the measured
    coding gain (r = 0, once per transform); returns (seconds in the oracle,
    pixels of the sweep the task stands for)."""
    img, kind, r = args
    from oracle import pipeline as P
    t0 = time.perf_counter()
    if r:
        P.compress(img, kind, N, r)
        return time.perf_counter() - t0, img.size
    P.empirical_coding_gain(img, kind, N, "cols")
    return time.perf_counter() - t0, 0


def cpu_baseline(pool, sample):
    """The oracle as it stands, timed on the host's cores over a bounded
    sample of the step: for every image of ``sample`` (drawn before the timed
    region) the full 14-point T x r sweep (compress with PSNR) and the measured
    coding gain of both transforms, one task per (image, T, r) pass or (image,
    T) gain.  ``value`` is pixels over the wall time of the oracle tasks; the
    summed time inside the oracle is reported beside it."""
    tasks = [(img, k, r) for img in sample for k in KINDS for r in (0,) + SWEEP_R]
    t0 = time.perf_counter()
    res = pool.map(_oracle_task, tasks)
    wall = time.perf_counter() - t0
    px = sum(p for _, p in res)
    cpu_s = sum(t for t, _ in res)
    h, w = sample[0].shape
    return {"value": px / wall / 1e9, "unit": "Gpixel/s", "cores": pool.workers,
            "kind": "oracle",
            "sample": f"{len(sample)} images of {h}x{w} from the same batch, the whole step: "
                      f"T x r sweep ({len(sample) * len(KINDS) * len(SWEEP_R)} passes, "
                      f"{px / 1e9:.2f} Gpx) and the coding gain of both T: {cpu_s:.1f} s "
                      f"inside the oracle over {pool.workers} {pool.kind}, {wall:.2f} s wall",
            "oracle_seconds": round(cpu_s, 2), "wall_seconds": round(wall, 3),
            "workers": pool.kind, "host_cpus": os.cpu_count(),
            "cpu_model": cpu_model()}


def cpu_model():
    """The host CPU's model name (first processor entry), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ------------------------------------------------------------------ GPU leg
def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("c0", "c1", "c2", "c3", "c4", "plain", "ceiling",
                                           "sweep", "compression"),
                    default="c1",
                    help="c0: latency of one 512^2 image; "
                         "c1: the 1024 x 2048^2 sweep (default; the line also carries the "
                         "ragged batch against per-image launches and the serving latency); "
                         "c2: the int16 residual frames with 16/32-point transforms and "
                         "quantisation; c3: the ragged batch alone; c4: the serving loop alone; "
                         "plain: one fused configuration (--n, --transform, --r, --qstep); "
                         "ceiling: the HBM read/write/copy ceilings of plain 16-byte kernels; "
                         "sweep: the transform assessment of section 4.1 (error energy, "
                         "deviation from diagonality, coding gain minus the KLT's over rho); "
                         "compression: the still-image experiment of section 5.1 (mean "
                         "PSNR and SSIM and their APE against the exact DCT for r = 1..45)")
    ap.add_argument("--engine", choices=("butterfly", "mfma"), default="butterfly",
                    help="c1/plain: N=8 uint8 zonal passes on the butterflies or on the int8 "
                         "matrix cores")
    ap.add_argument("--rate", type=float, default=2000.0, help="c4: arrivals per second")
    ap.add_argument("--duration", type=float, default=None,
                    help="c4: trace length in s (30 for --workload c4, 10 in the default line)")
    ap.add_argument("--pool", type=int, default=64, help="c4: device-resident images")
    ap.add_argument("--check-max", type=int, default=300,
                    help="c4: at most this many sampled requests checked against the oracle")
    ap.add_argument("--budget-gb", type=float, default=32.0, help="c4: HBM admission budget")
    ap.add_argument("--sweep", type=str, default="8000,32000,128000,512000,1000000",
                    help="c4: further arrival rates (1 s traces each), '' for none")
    ap.add_argument("--n", type=int, default=8)
    ap.add_argument("--transform", type=int, default=2)
    ap.add_argument("--r", type=int, default=10)
    ap.add_argument("--qstep", type=int, default=0)
    ap.add_argument("--dtype", choices=("u8", "i16"), default="u8")
    ap.add_argument("--images", type=int, default=None)
    ap.add_argument("--c3-images", type=int, default=10000,
                    help="c1 line: images of the ragged batch leg")
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--c1-only", action="store_true",
                    help="c1: time the sweep alone (no ragged-batch or serving leg)")
    ap.add_argument("--gen-workers", type=int, default=None,
                    help="host workers for input generation and the oracle (default: the "
                         "CPUs available, at most 16; threads under a profiler)")
    ap.add_argument("--ceiling-footprint", action="store_true",
                    help="ceiling: also time the best read/write/copy form of the 4 GiB "
                         "sweep on buffers of 0.25 to 16 GiB")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy kernel first (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this "
                         "benchmark into the committed traffic summary, then exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if under_profiler():
        log("running under a profiler: host work uses threads, no worker processes")

    if args.workload == "c0":
        run_c0(args)
    elif args.workload == "c2":
        run_c2(args)
    elif args.workload == "c3":
        with HostPool(host_workers(args.gen_workers)) as pool:
            data = prepare_c3(args, pool, args.images or 10000)
        print(json.dumps(c3_line(args, data, gpu_c3(args, data))), flush=True)
    elif args.workload == "c4":
        with HostPool(host_workers(args.gen_workers)) as pool:
            data = prepare_c4(args, pool, args.duration or 30.0)
        print(json.dumps(c4_line(args, data, gpu_c4(args, data, sweep=True))), flush=True)
    elif args.workload == "plain":
        run_plain(args)
    elif args.workload == "ceiling":
        run_ceiling(args)
    elif args.workload == "sweep":
        run_sweep(args)
    elif args.workload == "compression":
        run_compression(args)
    else:
        run_c1(args)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_c1(args):
    """The default line: the C1 sweep, plus (unless --c1-only) the ragged batch
    against per-image launches and the serving loop's p50/p99.  Every host
    input and the oracle baseline are prepared before the GPU is touched."""
    b, h, w = args.images or 1024, args.size, args.size
    extras = not args.c1_only
    t0 = time.perf_counter()
    with HostPool(host_workers(args.gen_workers)) as pool:
        imgs = c1_images(pool, b, h, w)
        log(f"generated {b} images of {h}x{w} in {time.perf_counter() - t0:.1f} s "
            f"({pool.workers} {pool.kind})")
        cpu = None
        if not args.no_cpu_baseline:
            cpu = cpu_baseline(pool, [imgs[i] for i in range(min(4, b))])
            log(f"CPU oracle: {cpu['value']:.3f} Gpx/s ({cpu['sample']})")
        c3 = prepare_c3(args, pool, args.c3_images) if extras else None
        c4 = prepare_c4(args, pool, args.duration or 10.0) if extras else None
    line = gpu_c1(args, imgs, cpu)
    if extras:
        r3 = gpu_c3(args, c3)
        line["batched_vs_plain"] = {
            "workload": c3["workload"], "graph_ms": r3["graph_ms"],
            "per_image_ms": r3["per_image_ms"], "speedup": r3["speedup"],
            "graph_gpixel_s": r3["graph_gpixel_s"],
            "per_image_gpixel_s": r3["per_image_gpixel_s"],
            "graph_hbm_frac": r3["roofline"]["frac"], "kernel": r3["roofline"]["kernel"],
            "parity_sample": r3["parity_sample"]}
        r4 = gpu_c4(args, c4, sweep=False)
        line["serving"] = {
            "workload": c4["workload"], "p50_ms": r4["main"]["p50_ms"],
            "p99_ms": r4["main"]["p99_ms"], "max_ms": r4["main"]["max_ms"],
            "served_gpixel_s": r4["main"]["served_gpixel_s"],
            "mean_batch": r4["main"]["mean_batch"],
            "host_wait_ms": r4["main"]["host_wait_ms"], "device_ms": r4["main"]["device_ms"],
            "slowest": r4["main"]["slowest"], "warmup_requests": r4["main"]["warmup_requests"],
            "cold_start_ms": r4["main"]["cold_start_ms"], "parity_sample": r4["parity_sample"]}
    print(json.dumps(line), flush=True)


def gpu_c1(args, imgs, cpu):
    import numpy as np
    import torch

    import paper_2207_11638_amd as adct
    import synth

    b, h, w = imgs.shape
    dev = gpu_device()
    x = torch.from_numpy(imgs).to(dev)
    tiles = b * (h // N) * (w // N)
    rmax = max(SWEEP_R)
    kept_buf = torch.empty(tiles * rmax, dtype=torch.int32, device=dev)
    scaled_buf = torch.empty(tiles * rmax, dtype=torch.float32, device=dev)
    recon = torch.empty_like(x)
    sse = torch.zeros(b, dtype=torch.uint64, device=dev)
    psnr = torch.zeros((len(KINDS), len(SWEEP_R), b), dtype=torch.float32, device=dev)
    mom = torch.zeros((len(KINDS), b, 3 * N * N + 4), dtype=torch.uint64, device=dev)
    cg = torch.zeros((len(KINDS), b), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    log("inputs resident on the GPU")

    if args.calibrate_copy:
        src = torch.ones(COPY_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.add(src, 0, out=dst)   # one elementwise kernel: reads and writes COPY_BYTES
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy done")

    combos = [(k, r) for k in KINDS for r in SWEEP_R]

    def views(r):
        return (kept_buf[: tiles * r].view(b, h // N, w // N, r),
                scaled_buf[: tiles * r].view(b, h // N, w // N, r))

    def one_step(events=None, mom_events=None):
        # per transform: the coefficient moments and the measured coding gain
        # (they do not depend on r), then the fused pass and PSNR of every r
        for ki, k in enumerate(KINDS):
            mom[ki].zero_()
            if mom_events is not None:
                mom_events[ki][0].record()
            adct.moments(x, k, N, out=mom[ki])
            if mom_events is not None:
                mom_events[ki][1].record()
            adct.coding_gain(mom[ki], k, N, "cols", out=cg[ki])
            for ri, r in enumerate(SWEEP_R):
                i = ki * len(SWEEP_R) + ri
                kv, sv = views(r)
                sse.zero_()
                if events is not None:
                    events[i][0].record()
                adct.compress(x, k, N, r, kept=kv, scaled=sv, recon=recon, sse=sse,
                              engine=args.engine)
                if events is not None:
                    events[i][1].record()
                adct.psnr(sse, h * w, out=psnr[ki, ri])

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    # events recorded on the current stream, the one the launches go to
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
           for _ in combos] for _ in range(args.steps)]
    mev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
            for _ in KINDS] for _ in range(args.steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for s in range(args.steps):
        one_step(ev[s], mev[s])
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    log(f"timed {args.steps} steps in {total_ms:.1f} ms")

    # per-launch durations of the fused kernel, averaged over steps
    per = {}
    for s in range(args.steps):
        for i, (k, r) in enumerate(combos):
            per.setdefault((k, r), []).append(ev[s][i][0].elapsed_time(ev[s][i][1]))
    kernels = []
    tot_bytes = tot_ms = 0.0
    for (k, r), ts in per.items():
        ms = sum(ts) / len(ts)
        by = algorithmic_bytes(b, h, w, r)
        tot_bytes += by
        tot_ms += ms
        kernels.append({"T": k, "r": r, "ms": round(ms, 4), "GBps": round(by / ms / 1e6, 1)})
    achieved = tot_bytes / tot_ms / 1e6   # GB/s, averaged over the 14 launches
    mom_ms = sum(mev[s][ki][0].elapsed_time(mev[s][ki][1])
                 for s in range(args.steps) for ki in range(len(KINDS))) / (args.steps * len(KINDS))
    moments_kernel = {"ms": round(mom_ms, 4), "GBps": round(b * h * w / mom_ms / 1e6, 1),
                      "bytes": "pixels read once, 8 B per coefficient sum per workgroup"}
    px_per_step = b * h * w * len(combos)
    value = px_per_step * args.steps / (total_ms / 1e3) / 1e9

    check = None
    if not args.no_check:
        from concurrent.futures import ThreadPoolExecutor

        from oracle import pipeline as P
        k, r = 2, 10
        kv, sv = views(r)
        sse.zero_()
        adct.compress(x, k, N, r, kept=kv, scaled=sv, recon=recon, sse=sse, engine=args.engine)
        torch.cuda.synchronize()
        picks = sorted({0, b // 2, b - 1})
        psnr_h = psnr.cpu().numpy().astype(np.float64)
        cg_h = cg.cpu().numpy().astype(np.float64)

        def near(got, want):
            return got == want or abs(got - want) <= 1e-5 * max(abs(want), 1.0)

        def one(i):
            want = P.compress(imgs[i], k, N, r)
            bad = int(not np.array_equal(kv[i].cpu().numpy(), want["kept"]))
            bad += int(not np.array_equal(recon[i].cpu().numpy(), want["recon"]))
            bad += int(int(sse[i].item()) != want["sse"])
            # PSNR and coding gain of the timed steps
            bad += int(not near(psnr_h[KINDS.index(k), SWEEP_R.index(r), i], want["psnr"]))
            for ki, kk in enumerate(KINDS):
                bad += int(not near(cg_h[ki, i], P.empirical_coding_gain(imgs[i], kk, N, "cols")))
            got_s = sv[i].cpu().numpy().astype(np.float64)
            nz = want["scaled"] != 0
            bad += int(not np.all(got_s[~nz] == 0))
            bad += int(not np.all(np.abs(got_s[nz] - want["scaled"][nz])
                                  <= 1e-5 * np.abs(want["scaled"][nz])))
            return bad

        with ThreadPoolExecutor(len(picks)) as ex:
            bad = sum(ex.map(one, picks))
        check = "ok" if bad == 0 else f"{bad} mismatches"
        log(f"sampled parity vs oracle (T2, r=10 outputs and PSNR, coding gain of T1 and T2; "
            f"images {picks}): {check}")

    traffic = measured_traffic() if args.engine == "butterfly" else None
    kernel = ("compress8 (fused 8x8 kernel; 14 instantiations, one per (T, r))"
              if args.engine == "butterfly" else
              "compress8_mfma (fused 8x8 kernel on the int8 matrix cores)")
    return {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded 2D AR(1) uint8 images)",
        "config": {"workload": f"plain method at scale: {b} x {h}x{w} uint8 AR(1) images, N=8, "
                               "T1+T2 x r in {1,6,10,16,28,45,64}, fused fwd+retain+scale+inv+SSE",
                   "images": b, "height": h, "width": w, "n": N, "r_sweep": list(SWEEP_R),
                   "outputs": "kept int32 + scaled float32 + recon uint8 + sse + float32 "
                              "PSNR per (T, r, image); coefficient moments + float32 measured "
                              "coding gain per (T, image)",
                   "engine": args.engine},
        "blocks_per_s": round(tiles * len(combos) * args.steps / (total_ms / 1e3), 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": kernel},
        "kernels": kernels,
        "moments_kernel": moments_kernel,
        "coding_gain_db": {f"T{k}": round(float(cg[ki].double().mean()), 4)
                           for ki, k in enumerate(KINDS)},
        "parity_sample": check,
        "cpu_baseline": cpu,
    }


# ------------------------------------------------- transform assessment sweep
def run_compression(args):
    """Section 5.1's still-image experiment on synthetic stand-ins: 30
    seeded 512 x 512 uint8 AR(1) images (rho 0.80 .. 0.98, one per image; the
    paper's 30 standard images are not available) compressed by every 8-point
    transform of the library and the exact DCT at r = 1..45.  Per (T, r): mean
    PSNR and mean SSIM over the images and the mean over the images of their
    absolute percentage errors against the exact DCT's (Figs. 3 and 4).  A
    sample is checked against the oracle."""
    import numpy as np
    import torch

    import paper_2207_11638_amd as adct
    import synth

    n_img = args.images or 30
    size = 512
    rhos = [0.80 + 0.18 * i / max(1, n_img - 1) for i in range(n_img)]
    imgs = [synth.ar1_image(size, size, rho=r_, seed=5100 + i) for i, r_ in enumerate(rhos)]
    dev = gpu_device()
    x = torch.from_numpy(np.stack(imgs)).to(dev)
    recon = torch.empty_like(x)
    sse = torch.zeros(n_img, dtype=torch.uint64, device=dev)
    names = {adct.ADCT_T1: "T1", adct.ADCT_T2: "T2", adct.ADCT_SDCT: "SDCT",
             adct.ADCT_WHT: "WHT", adct.ADCT_HT: "HT", adct.ADCT_DCT: "DCT"}
    rs = list(range(1, 46))
    psnr, ssim = {}, {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in names:
        for r in rs:
            sse.zero_()
            adct.compress(x, k, 8, r, kept=False, scaled=False, recon=recon, sse=sse)
            psnr[(k, r)] = adct.psnr(sse, size * size)
            ssim[(k, r)] = adct.ssim(x, recon)
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t0
    curves = {}
    for k, nm in names.items():
        c = {"psnr": [], "ssim": [], "psnr_ape": [], "ssim_ape": []}
        for r in rs:
            c["psnr"].append(round(float(psnr[(k, r)].mean()), 4))
            c["ssim"].append(round(float(ssim[(k, r)].mean()), 5))
            if k != adct.ADCT_DCT:
                c["psnr_ape"].append(round(float(
                    adct.ape(psnr[(k, r)], psnr[(adct.ADCT_DCT, r)]).mean()), 4))
                c["ssim_ape"].append(round(float(
                    adct.ape(ssim[(k, r)], ssim[(adct.ADCT_DCT, r)]).mean()), 4))
        curves[nm] = c
        log(f"{nm}: mean PSNR r=1 {c['psnr'][0]:.2f}, r=10 {c['psnr'][9]:.2f}, r=45 "
            f"{c['psnr'][44]:.2f} dB; mean SSIM r=10 {c['ssim'][9]:.4f}")
    # the orderings section 5.1 reports for the standard images; at r = 1 only
    # the DC coefficient is kept, the same for every transform
    p = {nm: np.array(curves[nm]["psnr"]) for nm in curves}
    orderings = {
        "r = 1: every transform equals the DCT": bool(all(p[nm][0] == p["DCT"][0] for nm in p)),
        "T2 PSNR above SDCT, 2 <= r <= 45": bool(np.all(p["T2"][1:] > p["SDCT"][1:])),
        "T2 PSNR above WHT, 2 <= r <= 15": bool(np.all(p["T2"][1:15] > p["WHT"][1:15])),
        "T2 PSNR above T1, 2 <= r <= 45": bool(np.all(p["T2"][1:] > p["T1"][1:])),
        "HT PSNR below WHT, 2 <= r <= 45": bool(np.all(p["HT"][1:] < p["WHT"][1:])),
    }
    for kk, v in orderings.items():
        log(f"{kk}: {v}")
    check = None
    if not args.no_check:
        from oracle import metrics as Q
        from oracle import pipeline as P
        bad = 0
        recon_h = {}
        for k, r in ((adct.ADCT_T2, 5), (adct.ADCT_T1, 20), (adct.ADCT_WHT, 10),
                     (adct.ADCT_SDCT, 45), (adct.ADCT_DCT, 10)):
            sse.zero_()
            adct.compress(x, k, 8, r, kept=False, scaled=False, recon=recon, sse=sse)
            recon_h[(k, r)] = recon.cpu().numpy()
            for i in (0, n_img - 1):
                want = P.compress_dct(imgs[i], r) if k == adct.ADCT_DCT else \
                    P.compress(imgs[i], k, 8, r)
                # the float32 DCT may round a pixel whose float64 value lies
                # within 1e-2 of a tie the other way: compare it within 1e-4
                tol = 1e-4 if k == adct.ADCT_DCT else 1e-5
                got_p = float(psnr[(k, r)][i])
                bad += int(abs(got_p - want["psnr"]) > tol * abs(want["psnr"]))
                want_s = Q.mean_ssim(imgs[i], want["recon"])
                got_s = float(ssim[(k, r)][i])
                bad += int(abs(got_s - want_s) > tol * max(abs(want_s), 1.0))
                if k != adct.ADCT_DCT:
                    bad += int(not np.array_equal(recon_h[(k, r)][i], want["recon"]))
        check = "ok" if bad == 0 else f"{bad} mismatches"
        log(f"sampled parity vs oracle (5 (T, r) points, images 0 and {n_img - 1}: "
            f"reconstruction, PSNR, SSIM): {check}")
    print(json.dumps({"workload": "still-image compression of section 5.1: "
                                  f"{n_img} AR(1) 512x512 uint8 stand-ins, r = 1..45",
                      "images": n_img, "rho": [round(rhos[0], 3), round(rhos[-1], 3)],
                      "gpu_seconds": round(gpu_s, 3),
                      "passes": len(names) * len(rs),
                      "ape": "mean over images of 100 |m - m_DCT| / m_DCT",
                      "curves": curves, "orderings": orderings,
                      "parity_sample": check}), flush=True)


def run_sweep(args):
    """Section 4.1's assessment of every transform the library offers: the
    total error energy and the deviation from diagonality (host, float64) and
    the coding gain minus the KLT's under the AR(1) model for rho in [0, 1)
    (one GPU launch per transform over the whole rho grid, float32, columns
    basis).  A sample of the grid is checked against the oracle."""
    import numpy as np
    import torch

    import paper_2207_11638_amd as adct
    dev = gpu_device()
    rhos = np.concatenate([np.arange(0, 100) / 100.0, [0.995, 0.999]]).astype(np.float32)
    d_rho = torch.from_numpy(rhos).to(dev)
    combos = [(k, n) for k in (1, 2) for n in (8, 16, 32, 64)] + [(k, 8) for k in (3, 4, 5)]
    names = {1: "T1", 2: "T2", 3: "WHT", 4: "SDCT", 5: "HT"}
    rows, cg_all, klt_all = [], {}, {}
    t0 = time.perf_counter()
    for k, n in combos:
        cg, klt = adct.coding_gain_ar1(d_rho, k, n, "cols")
        cg_all[(k, n)], klt_all[(k, n)] = cg, klt
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t0
    for k, n in combos:
        eps, delta = adct.transform_measures(k, n)
        diff = (cg_all[(k, n)] - klt_all[(k, n)]).cpu().numpy().astype(np.float64)
        pick = {f"{r:.3f}": round(float(diff[i]), 4) for i, r in enumerate(rhos)
                if round(float(r), 3) in (0.5, 0.9, 0.95, 0.99)}
        rows.append({"transform": names[k], "n": n, "eps": round(eps, 4), "delta": round(delta, 4),
                     "cg_minus_klt_db": pick})
        log(f"{names[k]} N={n}: eps {eps:.4f}, delta {delta:.4f}, C_g - C_g(KLT) {pick}")
    check = None
    if not args.no_check:
        from oracle import matrices as M
        from oracle import metrics as Q
        bad = 0
        for k, n in combos:
            c = M.near_orthogonal(k, n)
            cg = cg_all[(k, n)].cpu().numpy()
            kl = klt_all[(k, n)].cpu().numpy()
            for i in range(0, len(rhos), 7):
                r = float(rhos[i])
                for got, want in ((cg[i], Q.coding_gain(c, r, "cols")),
                                  (kl[i], Q.klt_coding_gain(n, r))):
                    bad += int(abs(float(got) - want) > 1e-5 * max(abs(want), 1.0))
        check = "ok" if bad == 0 else f"{bad} mismatches"
        log(f"sampled parity vs oracle (every 7th rho, every transform): {check}")
    print(json.dumps({"workload": "transform assessment of section 4.1 over rho in [0, 1)",
                      "rho_values": len(rhos), "gpu_seconds": round(gpu_s, 4),
                      "basis": "columns of C^-1", "transforms": rows,
                      "parity_sample": check}), flush=True)


# ------------------------------------------------------------ HBM ceilings
CEILING_BYTES = 4 << 30


def run_ceiling(args):
    """Read-only, write-only and copy streams of 4 GiB through the library's
    plain 16-byte non-temporal kernels (adct_stream_ceiling), over a sweep of
    grid sizes and loads in flight; each point timed with HIP events on the
    launch stream over --steps launches after --warmup.  Prints the best rate
    of each pattern (bytes moved: read, written, or both for the copy)."""
    import ctypes as C

    import torch

    from paper_2207_11638_amd import _lib
    lib = _lib.load()
    dev = gpu_device()
    src = torch.zeros(CEILING_BYTES, dtype=torch.uint8, device=dev)
    dst = torch.empty(CEILING_BYTES, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    sp = C.c_void_p(stream.cuda_stream)
    results = {}
    for pattern, name, moved in ((0, "read", 1), (1, "write", 1), (2, "copy", 2),
                                 (3, "read_chunked", 1), (4, "write_chunked", 1),
                                 (5, "copy_chunked", 2)):
        best = None
        for blocks in (2048, 8192, 16384, 32768, 65536):
            for unroll in ((1,) if pattern == 1 else (1, 2, 4, 8)):
                def go():
                    _lib.check(lib.adct_stream_ceiling(pattern, C.c_void_p(dst.data_ptr()),
                                                       C.c_void_p(src.data_ptr()), CEILING_BYTES,
                                                       blocks, unroll, sp))
                for _ in range(max(1, args.warmup)):
                    go()
                a = torch.cuda.Event(enable_timing=True)
                z = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(args.steps):
                    go()
                z.record(stream)
                torch.cuda.synchronize()
                ms = a.elapsed_time(z) / args.steps
                gbs = moved * CEILING_BYTES / ms / 1e6
                log(f"{name}: {blocks} workgroups, {unroll} in flight: {ms:.3f} ms, {gbs:.0f} GB/s")
                if best is None or gbs > best["GBps"]:
                    best = {"GBps": round(gbs, 1), "ms": round(ms, 4), "workgroups": blocks,
                            "unroll": unroll}
        results[name] = best
    footprint = None
    if args.ceiling_footprint:
        # the best form of each pattern on smaller and larger buffers (one
        # 16 GiB pair at most: 32 GiB of the 288 GB)
        del src, dst
        torch.cuda.empty_cache()
        footprint = {}
        for gib in (0.25, 1, 2, 4, 8, 16):
            nbytes = int(gib * (1 << 30))
            src = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
            dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            row = {}
            for pattern, name, moved in ((0, "read", 1), (1, "write", 1), (2, "copy", 2),
                                         (3, "read_chunked", 1), (4, "write_chunked", 1),
                                         (5, "copy_chunked", 2)):
                best = results[name]

                def go():
                    _lib.check(lib.adct_stream_ceiling(pattern, C.c_void_p(dst.data_ptr()),
                                                       C.c_void_p(src.data_ptr()), nbytes,
                                                       best["workgroups"], best["unroll"], sp))
                for _ in range(max(1, args.warmup)):
                    go()
                a = torch.cuda.Event(enable_timing=True)
                z = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(args.steps):
                    go()
                z.record(stream)
                torch.cuda.synchronize()
                ms = a.elapsed_time(z) / args.steps
                row[name] = round(moved * nbytes / ms / 1e6, 1)
            log(f"footprint {gib} GiB per buffer: {row}")
            footprint[str(gib)] = row
            del src, dst
            torch.cuda.empty_cache()
    print(json.dumps({"workload": "HBM streaming ceilings, 4 GiB per buffer, 16-byte "
                                  "non-temporal accesses", "peak_GBps": HBM_PEAK_GBS,
                      "ceilings": results,
                      "fraction_of_peak": {k: round(v["GBps"] / HBM_PEAK_GBS, 4)
                                           for k, v in results.items()},
                      "footprint_GBps": footprint}), flush=True)


# ---------------------------------------------------------------- one config
def run_plain(args):
    """One fused configuration over a batch of equal images (uint8 AR(1) or
    int16 Laplacian residuals), outputs kept + scaled + recon + sse."""
    import numpy as np
    import torch

    import paper_2207_11638_amd as adct
    import synth

    b, h, w, n, r = args.images or 256, args.size, args.size, args.n, args.r
    if args.dtype == "u8":
        with HostPool(host_workers(args.gen_workers)) as pool:
            imgs = c1_images(pool, b, h, w)
    else:
        imgs = np.stack([synth.laplace_residual(h, w, seed=2000 + i) for i in range(b)])
    dev = gpu_device()
    x = torch.from_numpy(imgs).to(dev)
    tiles = b * (h // n) * (w // n)
    kept = torch.empty((b, h // n, w // n, r), dtype=torch.int32, device=dev)
    scaled = torch.empty((b, h // n, w // n, r), dtype=torch.float32, device=dev)
    recon = torch.empty_like(x)
    sse = torch.zeros(b, dtype=torch.uint64, device=dev)

    def step():
        adct.compress(x, args.transform, n, r, args.qstep, kept=kept, scaled=scaled, recon=recon,
                      sse=sse, engine=args.engine)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    z = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        step()
    z.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(z) / args.steps
    esize = x.element_size()
    algo = b * h * w * 2 * esize + tiles * r * 8 + b * 8
    achieved = algo / ms / 1e6
    print(json.dumps({"metric": METRIC, "value": round(b * h * w / ms / 1e6, 2),
                      "unit": "Gpixel/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": round(ms, 4),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "int32", "data": "synthetic",
                      "config": {"workload": f"plain: {b} x {h}x{w} {args.dtype}, N={n}, "
                                             f"T{args.transform}, r={r}, qstep={args.qstep}"},
                      "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
                      "cpu_baseline": None}), flush=True)


# --------------------------------------------------------------- ragged batch
def run_c0(args):
    """One 512 x 512 AR(1) image (rho 0.95, sigma 40, seed 0), N = 8, r = 10,
    T1 and T2: the fused compress of one image (kept, scaled, recon, sse) is
    cache-resident, so it is reported as latency: the median and 99th
    percentile over repeated single launches, each bracketed by events, and
    checked bit-exact against the oracle."""
    import numpy as np
    import torch

    import paper_2207_11638_amd as adct
    import synth

    img = synth.ar1_image(512, 512, rho=0.95, sigma=40.0, seed=0)
    dev = gpu_device()
    x = torch.from_numpy(img).to(dev)[None]
    reps = max(200, 50 * args.steps)
    res = {}
    check = "ok"
    for kind in (1, 2):
        outs = adct.compress(x, kind, 8, 10)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, z in ev:
            a.record()
            adct.compress(x, kind, 8, 10, kept=outs["kept"], scaled=outs["scaled"],
                          recon=outs["recon"], sse=outs["sse"])
            z.record()
        torch.cuda.synchronize()
        us = np.array([a.elapsed_time(z) * 1e3 for a, z in ev])
        res[f"T{kind}"] = {"p50_us": round(float(np.percentile(us, 50)), 2),
                           "p99_us": round(float(np.percentile(us, 99)), 2)}
        if not args.no_check:
            from oracle import pipeline as P
            want = P.compress(img, kind, 8, 10)
            outs["sse"].zero_()
            adct.compress(x, kind, 8, 10, kept=outs["kept"], scaled=outs["scaled"],
                          recon=outs["recon"], sse=outs["sse"])
            torch.cuda.synchronize()
            ok = (np.array_equal(outs["kept"][0].cpu().numpy(), want["kept"])
                  and np.array_equal(outs["recon"][0].cpu().numpy(), want["recon"])
                  and int(outs["sse"][0].item()) == want["sse"])
            if not ok:
                check = "mismatch"
    p50 = max(v["p50_us"] for v in res.values())
    log(f"latency per image: {res}; oracle check {check}")
    print(json.dumps({
        "metric": METRIC, "value": round(512 * 512 / p50 / 1e3, 3), "unit": "Gpixel/s",
        "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": round(p50 / 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded 2D AR(1) uint8 image)",
        "config": {"workload": "one 512x512 uint8 AR(1) image (rho 0.95, seed 0), N=8, r=10, "
                               "T1 and T2: single-launch latency"},
        "latency_us": res, "roofline": None, "parity_sample": check, "cpu_baseline": None,
    }), flush=True)


def _c2_frame(f):
    import synth
    return synth.residual_frame_planes(f)


def run_c2(args):
    """64 int16 residual frames (3840 x 2160 luma + two 1920 x 1080 chroma
    planes, i.i.d. Laplacian with scale 12 clipped to [-255, 255], plane p of
    frame f from seed 2000 + 3 f + p).  One step = 16 passes over all frames:
    N in {16, 32} x T in {T1, T2} x Q in {8, 16, 32, 64}, every coefficient
    quantised (r = N^2), levels int32 + reconstruction int16 + error energy.
    Heights 2160 and 1080 are not multiples of 32 (1080 not of 16): each
    plane is tiled by N x N units whose border strips are covered by the
    largest smaller TUs (the implicit split), through the TU-list path."""
    import numpy as np
    import torch

    import paper_2207_11638_amd as adct
    import synth
    from paper_2207_11638_amd import ragged

    frames = args.images or 64
    t0 = time.perf_counter()
    with HostPool(host_workers(args.gen_workers)) as pool:
        planes = [p for fr in pool.map(_c2_frame, range(frames)) for p in fr]
    dev = gpu_device()
    npx = sum(p.size for p in planes)
    log(f"generated {frames} frames ({len(planes)} planes, {npx / 1e6:.0f} Mpx) in "
        f"{time.perf_counter() - t0:.1f} s")
    configs = [(n, k, q) for n in (16, 32) for k in (1, 2) for q in (8, 16, 32, 64)]
    arena, base = ragged.pack_images(planes, [1] * len(planes), [1] * len(planes),
                                     [0] * len(planes))
    tu_tables = {n: ragged.tu_table([synth.quadtree_tus_fast(p.shape[0], p.shape[1],
                                                             synth.rng_for(0), p_split=0.0,
                                                             ctu=n)
                                     for p in planes]) for n in (16, 32)}
    plans = {}
    t0 = time.perf_counter()
    for n, k, q in configs:
        d = base.copy()
        d["transform"], d["r"], d["qstep"] = k, n * n, q
        plans[(n, k, q)] = adct.BatchPlan(d, tu_tables[n], torch.int16)
    log(f"{len(plans)} plans built in {time.perf_counter() - t0:.1f} s "
        f"({len(tu_tables[16])} / {len(tu_tables[32])} TUs per pass at N = 16 / 32)")
    src = torch.from_numpy(arena).to(dev)
    dst = torch.zeros_like(src)
    words = max(pl.kept_words for pl in plans.values())
    kept = torch.empty(words, dtype=torch.int32, device=dev)
    sse = torch.zeros(len(planes), dtype=torch.uint64, device=dev)
    psnr = torch.zeros(len(planes), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    for i, (c, pl) in enumerate(plans.items()):
        chosen = pl.tune(src, dst, kept, None, sse)
        log(f"tuned plan {i + 1}/{len(plans)} {c}: shapes {chosen.tolist()} "
            f"({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()

    def step(events=None):
        for i, c in enumerate(configs):
            if events is not None:
                events[i][0].record()
            plans[c].run(src, dst, kept, None, sse, psnr, mode="batched")
            if events is not None:
                events[i][1].record()

    for _ in range(args.warmup):
        step()
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
           for _ in configs] for _ in range(args.steps)]
    a = torch.cuda.Event(enable_timing=True)
    z = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for s_ in range(args.steps):
        step(ev[s_])
    z.record()
    torch.cuda.synchronize()
    total_ms = a.elapsed_time(z)
    per = []
    for i, (n, k, q) in enumerate(configs):
        ms = sum(ev[s_][i][0].elapsed_time(ev[s_][i][1]) for s_ in range(args.steps)) / args.steps
        per.append({"n": n, "T": k, "q": q, "ms": round(ms, 4),
                    "GBps": round((8 * npx + 16 * len(planes)) / ms / 1e6, 1)})
    pass_ms = [p_["ms"] for p_ in per]
    algo = (8 * npx + 16 * len(planes)) * len(configs)
    achieved = algo / sum(pass_ms) / 1e6
    log(f"timed {args.steps} steps in {total_ms:.1f} ms; per pass "
        f"{min(pass_ms):.2f}..{max(pass_ms):.2f} ms")

    check = None
    if not args.no_check:
        from oracle import pipeline as P
        bad = checked = 0
        rng = synth.rng_for(2999)
        for c in ((32, 2, 16), (16, 1, 64)):
            pl = plans[c]
            sse.zero_()
            pl.run(src, dst, kept, None, sse, psnr, mode="batched")
            torch.cuda.synchronize()
            dst_h, kept_h = dst.cpu().numpy(), kept.cpu().numpy()
            sse_h = sse.cpu().numpy().astype(np.int64)
            tut = tu_tables[c[0]]
            recs = {}
            for t in rng.choice(len(tut), size=400, replace=False):
                i, x, y, nn = (int(tut[t][f]) for f in ("image", "x", "y", "n"))
                out = P.compress(planes[i][y:y + nn, x:x + nn], c[1], nn, nn * nn, c[2])
                o = int(pl.tu_kept_offset[t])
                if i not in recs:
                    recs[i] = ragged.unpack_image(dst_h, pl.images[i])
                rec = recs[i]
                bad += int(not np.array_equal(kept_h[o:o + nn * nn], out["kept"].reshape(-1)))
                bad += int(not np.array_equal(rec[y:y + nn, x:x + nn], out["recon"]))
                checked += 1
            for i in (0, len(planes) - 1):   # error energy of whole planes, exact
                rec = ragged.unpack_image(dst_h, pl.images[i]).astype(np.int64)
                bad += int(int(((rec - planes[i]) ** 2).sum()) != sse_h[i])
        check = "ok" if bad == 0 else f"{bad} mismatches"
        log(f"sampled parity vs oracle ({checked} TUs of 2 configurations, plane error "
            f"energies): {check}")

    out = {
        "metric": METRIC,
        "value": round(npx * len(configs) * args.steps / total_ms / 1e6, 2),
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded i.i.d. Laplacian int16 residual frames, 4:2:0)",
        "config": {"workload": f"residual frames: {frames} x (3840x2160 + 2 x 1920x1080) int16, "
                               "N in {16,32} x T1/T2 x Q in {8,16,32,64}, all coefficients "
                               "quantised, implicit split at 2160/1080",
                   "frames": frames, "pixels_per_pass": npx, "passes": len(configs)},
        "passes": per,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "bucket_jam / bucket8 (int16, quantiser; tuned per-bucket "
                               "launches: one TU size dominates, so the unified launch's "
                               "lower occupancy does not pay)"},
        "parity_sample": check,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def _c3_image(job):
    import synth
    h, w, seed, rho = job
    return synth.ar1_arena_image(h, w, seed, rho)


def prepare_c3(args, pool, n):
    """Host side of the ragged batch: n images with log-normal sides in
    [64, 4096] (multiples of 8), AR(1) content with rho ~ U[0.85, 0.98], each
    split by a seeded HEVC-style quadtree (32x32 units, split probability 0.4
    per level, forced splits at the border) into 8/16/32 TUs; T1/T2 alternate
    by image, r ~ U{6..28} per image."""
    import numpy as np

    import paper_2207_11638_amd as adct
    import synth
    from paper_2207_11638_amd import ragged

    t0 = time.perf_counter()
    sizes = synth.ragged_sizes(n, seed=3000)
    hs, ws = sizes[:, 0], sizes[:, 1]
    rhos = np.array([synth.rng_for(1_003_000 + i).uniform(0.85, 0.98) for i in range(n)])
    pitches = (ws + 15) // 16 * 16
    offsets = np.zeros(n, dtype=np.int64)
    off = 0
    for i in range(n):
        off = (off + 255) // 256 * 256
        offsets[i] = off
        off += int(pitches[i] * hs[i])
    total = (off + 255) // 256 * 256
    arena = np.zeros(total, dtype=np.uint8)
    jobs = [(int(hs[i]), int(ws[i]), 3000 + i, float(rhos[i])) for i in range(n)]
    for i, img in enumerate(pool.imap(_c3_image, jobs, chunksize=8)):
        arena[offsets[i]:offsets[i] + pitches[i] * hs[i]].reshape(hs[i], pitches[i])[:, :ws[i]] = img
    rs = synth.rng_for(3002).integers(6, 29, size=n)
    descs = np.zeros(n, dtype=adct.IMAGE_DESC)
    descs["src_offset"] = offsets
    descs["dst_offset"] = offsets
    descs["height"], descs["width"], descs["pitch"] = hs, ws, pitches
    descs["transform"] = 1 + np.arange(n) % 2
    descs["r"] = rs
    tus = ragged.tu_table([synth.quadtree_tus_fast(int(hs[i]), int(ws[i]),
                                                   synth.rng_for(4_000_000 + i))
                           for i in range(n)])
    npx = int((hs * ws).sum())
    log(f"generated {n} ragged images ({npx / 1e9:.2f} Gpx) and {len(tus)} TUs in "
        f"{time.perf_counter() - t0:.1f} s")
    return {"n": n, "arena": arena, "descs": descs, "tus": tus, "npx": npx, "hs": hs, "ws": ws,
            "rs": rs, "offsets": offsets, "pitches": pitches,
            "workload": f"ragged batch: {n} AR(1) images ({npx / 1e9:.2f} Gpx), sides "
                        "log-normal in [64, 4096], 8/16/32 quadtree TUs (p=0.4), T1/T2, "
                        "r in 6..28"}


def gpu_c3(args, d):
    """One step = one pass over every TU (retained int32 coefficients,
    reconstruction, error energy and PSNR per image).  Timed four ways: one
    launch per bucket, the unified launch, its graph replay (the batched
    form), and one launch per image and bucket (the per-image baseline)."""
    import numpy as np
    import torch

    import paper_2207_11638_amd as adct
    from paper_2207_11638_amd import ragged

    n, npx, descs, tus = d["n"], d["npx"], d["descs"], d["tus"]
    dev = gpu_device()
    t0 = time.perf_counter()
    plan = adct.BatchPlan(descs, tus, torch.uint8)
    info = plan.info()
    log(f"plan built in {time.perf_counter() - t0:.1f} s: {info}")
    src = torch.from_numpy(d["arena"]).to(dev)
    dst = torch.zeros_like(src)
    kept = torch.empty(max(1, plan.kept_words), dtype=torch.int32, device=dev)
    sse = torch.zeros(n, dtype=torch.uint64, device=dev)
    psnr = torch.zeros(n, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    chosen = plan.tune(src, dst, kept, None, sse)
    log(f"tuned workgroup sizes per bucket: {chosen.tolist()}")

    def timed(mode, steps, warmup, stream=None):
        ctx = torch.cuda.stream(stream) if stream is not None else None
        if ctx:
            ctx.__enter__()
        try:
            for _ in range(warmup):
                plan.run(src, dst, kept, None, sse, psnr, mode=mode)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            z = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                plan.run(src, dst, kept, None, sse, psnr, mode=mode)
            z.record()
            torch.cuda.synchronize()
            return a.elapsed_time(z) / steps
        finally:
            if ctx:
                ctx.__exit__(None, None, None)

    ms_batched = timed("batched", args.steps, args.warmup)
    ms_unified = timed("unified", args.steps, args.warmup)
    ms_graph = timed("graph", args.steps, max(1, args.warmup), torch.cuda.Stream())
    ms_per_image = timed("per_image", 1, 1)
    log(f"ms per pass: batched {ms_batched:.2f}, unified {ms_unified:.2f}, graph {ms_graph:.2f}, "
        f"per-image launches {ms_per_image:.2f}")

    check = None
    if not args.no_check:
        from concurrent.futures import ThreadPoolExecutor

        from oracle import pipeline as P
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):   # graph capture needs a non-null stream
            plan.run(src, dst, kept, None, sse, psnr, mode="graph")
        torch.cuda.synchronize()
        dst_h = dst.cpu().numpy()
        kept_h = kept.cpu().numpy()
        sse_h = sse.cpu().numpy().astype(np.int64)
        psnr_h = psnr.cpu().numpy().astype(np.float64)
        arena = d["arena"]

        def one(i):
            h, w, o, pitch = (int(d[k][i]) for k in ("hs", "ws", "offsets", "pitches"))
            img = arena[o:o + pitch * h].reshape(h, pitch)[:, :w]
            rec = ragged.unpack_image(dst_h, descs[i])
            bad = e = 0
            for t in np.nonzero(tus["image"] == i)[0]:
                x, y, nn = int(tus[t]["x"]), int(tus[t]["y"]), int(tus[t]["n"])
                r = min(int(d["rs"][i]), nn * nn)
                out = P.compress(img[y:y + nn, x:x + nn], int(descs[i]["transform"]), nn, r)
                o_ = int(plan.tu_kept_offset[t])
                bad += int(not np.array_equal(kept_h[o_:o_ + r], out["kept"].reshape(-1)))
                bad += int(not np.array_equal(rec[y:y + nn, x:x + nn], out["recon"]))
                e += out["sse"]
            bad += int(e != sse_h[i])
            want_p = P.psnr(e, h * w)
            bad += int(not (want_p == psnr_h[i] or
                            abs(psnr_h[i] - want_p) <= 1e-5 * abs(want_p)))
            return bad

        picks = sorted({0, n // 2, n - 1})
        with ThreadPoolExecutor(len(picks)) as ex:
            bad = sum(ex.map(one, picks))
        check = "ok" if bad == 0 else f"{bad} mismatches"
        log(f"sampled parity vs oracle (graph replay; images {picks}, every TU, error "
            f"energy, PSNR): {check}")

    algo = 2 * npx + 4 * plan.kept_words + 12 * n
    achieved = algo / ms_graph / 1e6
    return {"batched_ms": round(ms_batched, 3), "unified_ms": round(ms_unified, 3),
            "graph_ms": round(ms_graph, 3), "per_image_ms": round(ms_per_image, 3),
            "speedup": round(ms_per_image / ms_graph, 2),
            "graph_gpixel_s": round(npx / ms_graph / 1e6, 2),
            "per_image_gpixel_s": round(npx / ms_per_image / 1e6, 2),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": None,
                         "kernel": ("bucket_unified_small" if info.get("small_bound") else
                                    "bucket_unified") + " (graph replay of one launch over all "
                                   "buckets, XCD-sliced item order)"},
            "plan": info, "tuned_block_sizes": chosen.tolist(), "parity_sample": check}


def c3_line(args, d, r):
    return {
        "metric": METRIC, "value": r["graph_gpixel_s"], "unit": "Gpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["graph_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded ragged AR(1) uint8 images, quadtree TUs)",
        "config": {"workload": d["workload"], "images": d["n"], "tus": int(len(d["tus"])),
                   "pixels": d["npx"]},
        "batched_vs_per_image": {k: r[k] for k in ("batched_ms", "unified_ms", "graph_ms",
                                                   "per_image_ms", "speedup",
                                                   "per_image_gpixel_s")},
        "roofline": r["roofline"], "plan": r["plan"], "tuned_block_sizes": r["tuned_block_sizes"],
        "parity_sample": r["parity_sample"], "cpu_baseline": None}


# -------------------------------------------------------------------- serving
def _c4_image(job):
    import synth
    h, w, seed, rho = job
    return synth.ar1_arena_image(h, w, seed, rho)


def prepare_c4(args, pool, duration):
    """Host side of the serving loop: a Poisson trace at --rate requests/s for
    ``duration`` s (seed 4000); each request is one image from a pool of
    --pool AR(1) images (sides log-normal around 1024 in [64, 4096],
    multiples of 32) with its own T in {T1, T2}, N in {8, 16, 32} and
    r in 6..28."""
    import numpy as np

    import synth

    n_req = int(args.rate * duration)
    trace = synth.serving_requests(n_req, seed=4000, rate_hz=args.rate)
    pool_n = min(args.pool, n_req)
    sizes = np.array([(t["h"], t["w"]) for t in trace[:pool_n]], dtype=np.int64)
    px = sizes[:, 0] * sizes[:, 1]
    offsets = np.concatenate([[0], np.cumsum(px)[:-1]]).astype(np.int64)
    jobs = [(int(sizes[i, 0]), int(sizes[i, 1]), 5000 + i, 0.85 + 0.13 * ((i * 0.618) % 1.0))
            for i in range(pool_n)]
    t0 = time.perf_counter()
    arena = np.zeros(int(px.sum()), dtype=np.uint8)
    for i, img in enumerate(pool.imap(_c4_image, jobs)):
        arena[offsets[i]:offsets[i] + px[i]] = img.reshape(-1)
    log(f"serving pool of {pool_n} images ({px.sum() / 1e6:.1f} Mpx) generated in "
        f"{time.perf_counter() - t0:.1f} s")
    sweep = []
    for rate in [float(v) for v in args.sweep.split(",") if v.strip()]:
        sweep.append((rate, synth.serving_requests(int(rate), seed=4001, rate_hz=rate)))
    return {"trace": trace, "n_req": n_req, "duration": duration, "pool_n": pool_n,
            "sizes": sizes, "px": px, "offsets": offsets, "arena": arena, "sweep": sweep,
            "workload": f"serving: Poisson {args.rate:.0f} req/s for {duration:.0f} s "
                        f"({n_req} requests), sides log-normal (median 1024) in [64, 4096], "
                        f"T1/T2, N in {{8,16,32}}, r in 6..28, {args.budget_gb:.0f} GB budget"}


def _c4_check(task):
    """Oracle check of one served request."""
    import numpy as np

    from oracle import pipeline as P
    img, kind, n, r, kept, recon, sse = task
    want = P.compress(img, kind, n, r)
    return (np.array_equal(kept.reshape(want["kept"].shape), want["kept"])
            and np.array_equal(recon, want["recon"]) and int(sse) == want["sse"])


def gpu_c4(args, d, sweep):
    """Replays the trace in real time through the library's native loop
    (admission by the HBM budget, continuous batching over two batch slots).
    Reports p50/p99 latency (arrival to completion event) and served
    Gpixel/s, checks a sample of >= 1 % of the requests (at most --check-max)
    against the oracle, and with ``sweep`` raises the arrival rate towards
    saturation and times the same saturating requests issued one plain
    adct_compress call each."""
    import numpy as np
    import torch

    import paper_2207_11638_amd as adct

    trace, n_req, pool_n = d["trace"], d["n_req"], d["pool_n"]
    sizes, px, offsets, arena = d["sizes"], d["px"], d["offsets"], d["arena"]
    dev = gpu_device()
    d_arena = torch.from_numpy(arena).to(dev)
    pool = [d_arena[int(o):int(o) + int(p)].view(int(h), int(w))
            for o, p, (h, w) in zip(offsets, px, sizes)]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream
    budget = int(args.budget_gb * (1 << 30))
    pool_ptr = np.array([int(x.data_ptr()) for x in pool], dtype=np.uint64)

    def build(trace_, sample_every):
        m = len(trace_)
        j = np.arange(m) % pool_n
        recs = np.zeros(m, dtype=adct.REQUEST)
        recs["d_src"] = pool_ptr[j]
        recs["pitch"] = sizes[j, 1]
        recs["tag"] = np.arange(m)
        recs["transform"] = [t["transform"] for t in trace_]
        recs["n"] = [t["n"] for t in trace_]
        recs["r"] = [t["r"] for t in trace_]
        recs["dtype"] = adct.ADCT_U8
        recs["height"] = sizes[j, 0]
        recs["width"] = sizes[j, 1]
        return recs

    def check_records(trace_, recs, sample_every):
        """The sampled requests again, with pinned host buffers that receive
        their kept coefficients and reconstruction.  They run as a separate
        replay: a copy into host memory issued from the loop thread has
        blocked that thread for 6-10 ms about once per trace, which would
        stall the timed requests arriving meanwhile."""
        picks = list(range(0, len(trace_), sample_every))
        sub_ = recs[picks].copy()
        j = np.arange(len(trace_)) % pool_n
        checks = []
        for k, i in enumerate(picks):
            t = trace_[i]
            h, w = (int(v) for v in sizes[j[i]])
            h_kept = torch.empty((h // t["n"]) * (w // t["n"]) * t["r"],
                                 dtype=torch.int32).pin_memory()
            h_recon = torch.empty((h, w), dtype=torch.uint8).pin_memory()
            sub_["h_kept"][k] = h_kept.data_ptr()
            sub_["h_recon"][k] = h_recon.data_ptr()
            checks.append((i, int(j[i]), h_kept, h_recon))
        return sub_, checks

    def replay(trace_, rate, sample_every=0):
        recs = build(trace_, sample_every)
        arrival_ms = np.array([t["t"] for t in trace_]) * 1e3
        srv = adct.Server(budget, max_inflight=2, max_batch=1024, stream=stream)
        lat, batch, sse, launch = srv.run_trace(recs, arrival_ms, launch_times=True)
        st = srv.stats()
        srv.close()
        served_px = int(px[np.arange(len(trace_)) % pool_n].sum())
        span_s = (np.max(arrival_ms + lat) - arrival_ms[0]) / 1e3
        res = {"rate_hz": rate, "requests": len(trace_),
               "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "max_ms": round(float(np.max(lat)), 3),
               "served_gpixel_s": round(served_px / span_s / 1e9, 3),
               "offered_gpixel_s": round(served_px / (arrival_ms[-1] / 1e3) / 1e9, 3),
               "batches": int(st["batches"]), "largest_batch": int(st["max_batch"]),
               "mean_batch": round(len(trace_) / max(1, st["batches"]), 2),
               "budget_waits": int(st["refused"])}
        # where the time went: waiting on the host (arrival -> launch of the
        # request's batch) and on the device (launch -> completion event)
        host = launch - arrival_ms
        dev = lat - host
        res["host_wait_ms"] = {"p50": round(float(np.percentile(host, 50)), 3),
                               "p99": round(float(np.percentile(host, 99)), 3),
                               "max": round(float(np.max(host)), 3)}
        res["device_ms"] = {"p50": round(float(np.percentile(dev, 50)), 3),
                            "p99": round(float(np.percentile(dev, 99)), 3),
                            "max": round(float(np.max(dev)), 3)}
        checks = None
        if sample_every:
            # the check replay: sampled requests submitted at once, outputs
            # copied to the host; its error energies must equal the timed ones
            sub_, checks = check_records(trace_, recs, sample_every)
            srv = adct.Server(budget, max_inflight=2, max_batch=1024, stream=stream)
            _, _, sse_c = srv.run_trace(sub_, np.zeros(len(sub_)))
            srv.close()
            checks = [(i, jj, hk, hr, int(sse_c[k]), int(sse[i]))
                      for k, (i, jj, hk, hr) in enumerate(checks)]
        return res, checks, sse, lat, (host, dev, batch)

    # warm-up: one request of each (transform, n, r) of the trace through a
    # throw-away server.  The first launch of a kernel loads its code on the
    # launching thread (about 2 ms), which would stall the first requests of
    # the timed trace; a server warms its classes once at start-up.  The
    # warm-up's slowest request is reported as the cold start.
    recs_w = build(trace, 0)
    keys = np.stack([recs_w["transform"], recs_w["n"], recs_w["r"]], axis=1)
    first = np.sort(np.unique(keys, axis=0, return_index=True)[1])
    srv_w = adct.Server(budget, max_inflight=2, max_batch=1024, stream=stream)
    lat_w, _, _ = srv_w.run_trace(recs_w[first].copy(), np.zeros(len(first)))
    srv_w.close()
    cold_ms = round(float(np.max(lat_w)), 3)

    main_res, checks, sse, lat, (host, dev, batch) = replay(
        trace, args.rate, sample_every=max(1, min(100, n_req // max(1, args.check_max))))
    main_res["warmup_requests"] = int(len(first))
    main_res["cold_start_ms"] = cold_ms
    slow = np.argsort(lat)[-3:][::-1]
    main_res["slowest"] = [{"request": int(i), "arrival_ms": round(trace[i]["t"] * 1e3, 3),
                            "latency_ms": round(float(lat[i]), 3),
                            "host_wait_ms": round(float(host[i]), 3),
                            "device_ms": round(float(dev[i]), 3), "batch": int(batch[i])}
                           for i in slow]
    log(f"warm-up: {len(first)} requests, one per (T, N, r) of the trace; slowest {cold_ms} ms "
        f"(first launches)")
    log(f"served {n_req} requests at {args.rate:.0f}/s: p50 {main_res['p50_ms']} ms, "
        f"p99 {main_res['p99_ms']} ms, max {main_res['max_ms']} ms, "
        f"{main_res['served_gpixel_s']} Gpx/s, {main_res['batches']} batches; slowest "
        f"{main_res['slowest']}")

    check = None
    if not args.no_check:
        from concurrent.futures import ThreadPoolExecutor
        tasks = []
        same = all(sc == st for _, _, _, _, sc, st in checks)
        for i, j, hk, hr, sc, _ in checks:
            t = trace[i]
            img = arena[int(offsets[j]):int(offsets[j] + px[j])].reshape(int(sizes[j, 0]),
                                                                          int(sizes[j, 1]))
            tasks.append((img, t["transform"], t["n"], t["r"], hk.numpy().copy(),
                          hr.numpy().copy(), sc))
        with ThreadPoolExecutor(host_workers(args.gen_workers)) as ex:
            good = list(ex.map(_c4_check, tasks)) + [same]
        check = "ok" if all(good) else f"{len(good) - sum(good)} of {len(good)} mismatches"
        log(f"oracle check of {len(tasks)} sampled requests ({100 * len(tasks) / n_req:.1f} %): "
            f"{check}")

    sweep_res = []
    plain = None
    if sweep:
        for rate, tr in d["sweep"]:
            res, _, _, _, _ = replay(tr, rate)
            sweep_res.append(res)
            log(f"sweep {rate:.0f}/s: p50 {res['p50_ms']} ms, p99 {res['p99_ms']} ms, "
                f"served {res['served_gpixel_s']} of offered {res['offered_gpixel_s']} Gpx/s, "
                f"mean batch {res['mean_batch']}")
            if res["served_gpixel_s"] < 0.8 * res["offered_gpixel_s"]:
                break
        if d["sweep"]:
            plain = plain_per_request(d["sweep"][-1][1][:20000], pool, sizes, pool_n)
            log(f"the same requests as one plain adct_compress call each: "
                f"{plain['gpixel_s']} Gpx/s ({plain['requests']} requests in "
                f"{plain['seconds']} s)")
    return {"main": main_res, "sweep": sweep_res, "plain_per_request": plain,
            "parity_sample": check}


def plain_per_request(trace_, pool, sizes, pool_n):
    """Every request of a saturating trace as its own adct_compress call (the
    fused plain pipeline, outputs kept + recon + error energy), issued back to
    back on one stream through the C ABI: the unbatched baseline of the
    serving loop at saturation."""
    import ctypes as C

    import numpy as np
    import torch

    from paper_2207_11638_amd import _lib
    lib = _lib.load()
    dev = pool[0].device
    m = len(trace_)
    j = np.arange(m) % pool_n
    words = max((int(sizes[j[i], 0]) // t["n"]) * (int(sizes[j[i], 1]) // t["n"]) * t["r"]
                for i, t in enumerate(trace_))
    kept = torch.empty(words, dtype=torch.int32, device=dev)
    recon = torch.empty(int((sizes[:, 0] * sizes[:, 1]).max()), dtype=torch.uint8, device=dev)
    sse = torch.zeros(1, dtype=torch.uint64, device=dev)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    calls = []
    for i, t in enumerate(trace_):
        x = pool[j[i]]
        h, w = int(sizes[j[i], 0]), int(sizes[j[i], 1])
        calls.append((t["transform"], t["n"], t["r"], 0, C.c_void_p(x.data_ptr()), 0, 1, h, w,
                      w, h * w, C.c_void_p(kept.data_ptr()), None, C.c_void_p(recon.data_ptr()),
                      C.c_void_p(sse.data_ptr()), stream))
    fn = lib.adct_compress
    for c in calls[:100]:
        fn(*c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in calls:
        if fn(*c) != 0:
            _lib.check(-4)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    npx = int(sum(int(sizes[j[i], 0]) * int(sizes[j[i], 1]) for i in range(m)))
    return {"requests": m, "seconds": round(sec, 3), "gpixel_s": round(npx / sec / 1e9, 3)}


def c4_line(args, d, r):
    main = r["main"]
    return {
        "metric": METRIC, "value": main["served_gpixel_s"], "unit": "Gpixel/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(d["duration"] * 1e3, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded Poisson trace, pool of AR(1) uint8 images)",
        "config": {"workload": d["workload"], "pool_images": d["pool_n"]},
        "latency_ms": {"p50": main["p50_ms"], "p99": main["p99_ms"], "max": main["max_ms"]},
        "serving": main, "sweep": r["sweep"], "plain_per_request": r["plain_per_request"],
        "roofline": None, "parity_sample": r["parity_sample"], "cpu_baseline": None}


if __name__ == "__main__":
    main()
