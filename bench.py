#!/usr/bin/env python3
"""Benchmark of the fast adaptive bilateral filter on one MI355X.

A step is one pass of the whole fast filter over one synthetic image
already resident in HBM, issued as exactly the launches abf_fast makes:
window bounds (abf_minmax), then either the moment and range stages fused
in one kernel (abf_moments_range; abf_fast_fused() says where abf_fast
takes this path: the box kernel on the mixed path at small radii) or the
stack path, moment stack then range stage (abf_stack_moments or, where the
Gaussian tile kernel takes the bounds itself, abf_moment_stack in one
launch; then abf_range). Each stage is its own C-ABI call so that each
kernel can be timed on its own. The K timed steps alternate between two
streams, each with its own stack and output buffers, so two images are in
flight (one image's kernels fill the other's kernel tails and launch
gaps), with no events between the kernels. The same K steps then run on
one stream (the single-stream rate, reported beside the value) and once
more on one stream with HIP events around every kernel, which gives each
kernel's live duration (roofline) and the per-step device latency
(p50/p99). The mixed-precision path is the headline value; the all-FP64
path, the other path of each precision (stack where abf_fast fuses, fused
where it does not; the outputs are identical bit for bit) and the GPU brute
force are timed beside it. Before any step is counted, every path runs a
fixed PREWARM_STEPS untimed steps on top of --warmup (a kernel runs slower
in the first few hundred launches of a process).

The CPU legs run before the GPU is touched (so the worker processes fork
from a process without a HIP context): Algorithm 1 exactly as printed
(``oracle.fast_abf_literal``) timed on a band of image rows on one host
thread and on one band per host core at once (a pool of forked processes,
one thread each), and the value-of-record oracle on a random sample of
pixels, whose values give the parity of both GPU paths (all null with
--no-cpu-baseline). A short serving stream (continuous batching of mixed
requests, p50/p99 at three offered loads) runs after the filter timing
(--serving-requests 0 skips it).

Prints ONE JSON line (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpix/s fast-ABF mixed vs all-FP64 on GPU at max err≤0.05/255; p50/p99 latency"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector, TFLOP/s
DEFAULT_WORKLOAD = "voronoi4096_box5_n8"
PREWARM_STEPS = 300           # untimed steps per path before the counted warm-up
MAX_POOL = 16                 # host processes of the all-core CPU leg (at most one per core, and no more than 16)
N_STREAMS = 2                  # images in flight in the timed steps (default of --streams)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class one_host_thread:
    """Limits the numerical libraries to one host thread (the CPU oracle's
    baseline is quoted per core)."""

    def __enter__(self):
        try:
            from threadpoolctl import threadpool_limits
            self._ctx = threadpool_limits(1)
        except Exception:                      # pragma: no cover
            self._ctx = None
        return self

    def __exit__(self, *exc):
        if self._ctx is not None:
            self._ctx.__exit__(*exc)
        return False


def stage_model(h, w, kernel, R, N, prec_bytes, theta_given):
    """Algorithmic bytes and FP64 flops per launch for each kernel group.

    bytes: the inputs a kernel must read and the outputs it must write,
    once each (halo re-reads and intermediates are overhead, not counted).
    flops: the minimal FP64 arithmetic of the method's formulas.
    """
    px = h * w
    b = prec_bytes
    tb = 4 if theta_given else 4     # theta plane, or f when theta = f
    win = 2 * R + 1
    conv_flops = (4 * N * win) if kernel == "gaussian" else (4 * N)   # two separable passes
    shift_flops = N * (N + 1) + 2 * N + (N * N) // 2                  # Prop. 3 shift, scale, Legendre
    range_flops = (N + 1) * (N + 2) + 8 * (N + 1) + 20                # fit, recursion, T1/T2, t0/lambda
    return {
        "minmax": dict(bytes=px * (4 + 8), flops=0),
        "moments": dict(bytes=px * (4 + 8 + N * b), flops=px * (conv_flops + shift_flops)),
        # window bounds and moments in one kernel: f in; alpha, beta, a~ out
        "stack": dict(bytes=px * (4 + 8 + N * b), flops=px * (conv_flops + shift_flops)),
        "range": dict(bytes=px * (8 + N * b + tb + 4 + b), flops=px * range_flops),
        # fused: f, theta, sigma in, alpha and beta in (or, where the kernel
        # takes the bounds itself, out); g^ out (the stack never leaves the CU)
        "moments_range": dict(bytes=px * (4 + 8 + tb + 4 + b),
                              flops=px * (conv_flops + shift_flops + range_flops)),
    }


# The sources each timed stage's kernel is compiled from (its own file and
# the headers that file includes).
_MOMENT_SOURCES = ("moments.hip", "moments_common.h", "range_eval.h", "erfcx_weideman.h",
                   "abf_internal.h")
STAGE_SOURCES = {
    "minmax": ("minmax.hip", "abf_internal.h"),
    "moments": _MOMENT_SOURCES,
    "stack": _MOMENT_SOURCES,
    "moments_range": _MOMENT_SOURCES,
    "range": ("range.hip", "range_eval.h", "erfcx_weideman.h", "abf_internal.h"),
}


def stage_source_hash(stage: str) -> str:
    """First 16 hex digits of the SHA-256 over the sources of one stage's
    kernel (file names and contents, in the order of STAGE_SOURCES):
    identifies the kernel a stored counter reading was taken with."""
    import hashlib
    h = hashlib.sha256()
    for name in STAGE_SOURCES[stage]:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_1811_02308_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, stage: str):
    """HBM bytes per launch of the mixed path's `stage` kernel on `workload`
    from profiles/traffic.md (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by
    the device-copy calibration), or None when no reading exists or the
    stage's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.md")
    if not os.path.exists(path) or stage not in STAGE_SOURCES:
        return None
    src = stage_source_hash(stage)
    with open(path) as fh:
        for line in fh:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) == 9 and cells[0] == workload and cells[1] == stage:
                return int(float(cells[7])) if cells[8] == src else None
    return None


def _literal_band(job):
    """One row band of Algorithm 1 as printed (``oracle.fast_abf_literal``)
    on one host thread: the band plus R rows of halo on each side (so its
    rows equal the whole image's), returns the seconds taken."""
    f, th, sg, kernel, R, N, ss, y0, rows = job
    import oracle
    H = f.shape[0]
    lo, hi = max(0, y0 - R), min(H, y0 + rows + R)
    with one_host_thread():
        t0 = time.perf_counter()
        oracle.fast_abf_literal(f[lo:hi], None if th is None else th[lo:hi], sg[lo:hi], kernel, R,
                                N, sigma_s=ss)
        return time.perf_counter() - t0


def host_cores():
    """Cores this process may run on, and the pool size the all-core leg
    uses (at most MAX_POOL)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:                     # pragma: no cover
        n = os.cpu_count() or 1
    return n, max(1, min(n, MAX_POOL))


def cpu_legs(wl, cpu_seconds: float, literal_seconds: float):
    """The CPU oracle on the machine's host (see the module docstring). Returns
    (cpu_baseline dict, parity pixels (ys, xs), oracle values there)."""
    import multiprocessing as mp
    import numpy as np
    import oracle
    f, th, sg = wl["f"], wl["theta"], wl["sigma"]
    H, W = f.shape
    R, N, kernel, ss = wl["R"], wl["N"], wl["kernel"], wl["sigma_s"]
    visible, pool_n = host_cores()
    # literal route, one thread: size the band to about literal_seconds
    probe_rows = max(4, min(H, 16))
    t_probe = _literal_band((f, th, sg, kernel, R, N, ss, H // 2, probe_rows))
    rows = int(max(probe_rows, min(H // pool_n, literal_seconds / max(t_probe / probe_rows, 1e-9))))
    y0 = (H - rows) // 2
    t1 = _literal_band((f, th, sg, kernel, R, N, ss, y0, rows))
    rate1 = rows * W / t1 / 1e6
    # the same band size on every pool process at once (disjoint bands)
    starts = [min(H - rows, (i * H) // pool_n) for i in range(pool_n)]
    jobs = [(f, th, sg, kernel, R, N, ss, s, rows) for s in starts]
    ctx = mp.get_context("fork")
    with ctx.Pool(pool_n) as pool:
        pool.map(int, range(pool_n))           # processes started before the clock
        t0 = time.perf_counter()
        pool.map(_literal_band, jobs)
        tall = time.perf_counter() - t0
    rate_all = pool_n * rows * W / tall / 1e6
    # value-of-record route on random pixels: the parity reference
    rng = np.random.default_rng(7)
    with one_host_thread():
        probe = 4000
        py = np.concatenate([[0, 0, H - 1, H - 1], rng.integers(0, H, probe)])
        px = np.concatenate([[0, W - 1, 0, W - 1], rng.integers(0, W, probe)])
        oracle.fast_abf(f, th, sg, kernel, R, N, sigma_s=ss, pixels=(py[:64], px[:64]))
        t0 = time.perf_counter()
        pref = oracle.fast_abf(f, th, sg, kernel, R, N, sigma_s=ss, pixels=(py, px))
        per_px = (time.perf_counter() - t0) / len(py)
        m = int(max(probe, min(H * W, cpu_seconds / max(per_px, 1e-9))))
        sy, sx = rng.integers(0, H, m), rng.integers(0, W, m)
        t0 = time.perf_counter()
        sref = oracle.fast_abf(f, th, sg, kernel, R, N, sigma_s=ss, pixels=(sy, sx))
        dt = time.perf_counter() - t0
    cpu = {"value": round(rate_all, 4), "unit": "Mpix/s", "cores": pool_n, "kind": "oracle",
           "sample": f"Algorithm 1 as printed (FP64 NumPy, convolutions + binomial shift + integer "
                     f"A^-1 + erf/recursion) on {pool_n} disjoint {rows}-row bands of the same "
                     f"{H}x{W} workload at once, one process per core, one thread each, "
                     f"{tall:.1f} s",
           "single_core": {"value": round(rate1, 4), "unit": "Mpix/s", "cores": 1,
                           "sample": f"one {rows}-row band, one thread, {t1:.1f} s"},
           "host_cores_visible": visible,
           "value_of_record_route": {"value": round(m / dt / 1e6, 6), "unit": "Mpix/s", "cores": 1,
                                     "sample": f"{m} random pixels, one thread, {dt:.1f} s "
                                               f"(also the parity reference)"}}
    ys, xs = np.concatenate([py, sy]), np.concatenate([px, sx])
    return cpu, (ys, xs), np.concatenate([pref, sref])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # (1000 steps of the default 4096 x 4096 workload take about half a
    # second per path and stream configuration)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--streams", type=int, default=N_STREAMS,
                    help="streams the timed steps alternate between (1 for profiling: "
                         "kernels that overlap report stretched durations)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="seconds of the value-of-record oracle on sampled pixels (parity)")
    ap.add_argument("--literal-seconds", type=float, default=6.0,
                    help="seconds of one thread of the printed Algorithm 1 on its row band")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 256 MiB device-to-device copy (counter calibration for profiles)")
    ap.add_argument("--paper-maps", action="store_true",
                    help="the applications with the paper's parameter maps (sharpening, texture procedure)")
    ap.add_argument("--classical", action="store_true",
                    help="classical-filter sweep over rho and N (timing and PSNR tables) instead of the headline")
    ap.add_argument("--precision-table", action="store_true",
                    help="the 4096 x 4096 Voronoi precision sweep (box rho 5 and 20, N = 5..8): "
                         "mixed vs FP64 error per N instead of the headline")
    ap.add_argument("--kernel-sweep", action="store_true",
                    help="Gaussian tile kernel (O(rho) per pixel) vs the recursive kernel (O(1)) on a "
                         "4096 x 4096 field, N = 6, mixed, rho = 8..96, instead of the headline")
    ap.add_argument("--batched", action="store_true",
                    help="abf_fast_batched (one launch per stage per group) against one abf_fast call "
                         "per request, on small-image, mixed-size and 96-plane batches, instead of the headline")
    ap.add_argument("--serving-requests", type=int, default=400,
                    help="requests per offered load of the serving stream (p50/p99 at 3 loads); 0 skips it")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the filter runs on a single GPU (per-GPU sharding is described, not implemented); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np

    from synth import workload
    wl = None
    cpu, par_px, par_ref = None, None, None
    if args.precision_table:
        return precision_table(args)
    if args.kernel_sweep:
        return kernel_sweep(args)
    if args.batched:
        return batched_bench(args)
    if not (args.workload.startswith("texture") or args.classical or args.paper_maps):
        wl = workload(args.workload)
        if not args.no_cpu_baseline:
            log("CPU legs (printed Algorithm 1 on row bands; value-of-record oracle on sampled pixels) ...")
            cpu, par_px, par_ref = cpu_legs(wl, args.cpu_seconds, args.literal_seconds)

    import torch

    import paper_1811_02308_amd as abf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    abf.lib()
    if args.calibrate_copy:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    if args.workload.startswith("texture"):
        return texture_bench(args)
    if args.classical:
        return classical_bench(args)
    if args.paper_maps:
        return paper_maps_bench(args)
    f, th, sg = wl["f"], wl["theta"], wl["sigma"]
    H, W = f.shape
    R, N, kernel, ss = wl["R"], wl["N"], wl["kernel"], wl["sigma_s"]
    log(f"workload {args.workload}: {H}x{W} {kernel} R={R} N={N}")

    dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    fd, td, sd = dev(f), dev(th), dev(sg)

    single = abf.stack_single_pass(H, W, kernel, R, N)
    # the path abf_fast takes for each precision: bounds, then the moment and
    # range stages fused in one kernel, or the stack path
    fuses = {p: abf.fast_fused(H, W, kernel, R, N, p) for p in ("mixed", "fp64")}
    # the timed steps alternate between two streams, each with its own stack,
    # scratch and output buffers (two images in flight: one image's kernels
    # fill the other's kernel tails and launch gaps)
    n_streams = max(1, args.streams)
    streams = [torch.cuda.Stream() for _ in range(n_streams)]

    def make_path(prec, fused):
        # fused with a moment kernel that takes the window bounds itself (the
        # Gaussian tile kernel): abf_fast runs the whole filter as one kernel
        one = fused and single
        bufs = []
        for _ in range(n_streams):
            sb = (abf.workspace_bytes(H, W, R, N, prec, kernel) if one
                  else abf.stack_bytes(H, W, N, prec))
            bufs.append((torch.empty(sb, dtype=torch.uint8, device="cuda"),
                         torch.empty(abf.lib().abf_scratch_bytes(H, W, R), dtype=torch.uint8, device="cuda"),
                         torch.empty((H, W), dtype=torch.float32 if prec == "mixed" else torch.float64,
                                     device="cuda")))
        if one:
            names = ["moments_range"]
        elif fused:
            names = ["minmax", "moments_range"]
        else:
            names = ["stack", "range"] if single else ["minmax", "moments", "range"]

        def step(j=0, stream=None, ev=None):
            stack, scr, out = bufs[j]
            if ev is not None:
                ev[0].record()
            if one:
                abf.fast(fd, sd, theta=td, kernel=kernel, rho=R, N=N, sigma_s=ss, precision=prec,
                         out=out, workspace=stack, stream=stream)
                if ev is not None:
                    ev[1].record()
                return
            if fused or not single:
                abf.minmax_into_stack(fd, stack, R, N, prec, workspace=scr, stream=stream)
                if ev is not None:
                    ev[1].record()
            if fused:
                abf.moments_range(fd, stack, sd, theta=td, kernel=kernel, rho=R, N=N, sigma_s=ss,
                                  precision=prec, out=out, stream=stream)
            else:
                if single:
                    abf.moment_stack(fd, kernel=kernel, rho=R, N=N, sigma_s=ss, precision=prec,
                                     stack=stack, workspace=scr, stream=stream)
                else:
                    abf.stack_moments(fd, stack, kernel=kernel, rho=R, N=N, sigma_s=ss, precision=prec,
                                      stream=stream)
                if ev is not None:
                    ev[len(names) - 1].record()
                abf.range_from_stack(stack, sd, img=fd, theta=td, N=N, precision=prec, out=out,
                                     stream=stream)
            if ev is not None:
                ev[len(names)].record()

        return bufs, step, names

    def time_path(prec, steps, warmup, fused=False):
        bufs, step, names = make_path(prec, fused)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
               for _ in range(steps)]
        cur = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(cur)
        for i in range(PREWARM_STEPS + warmup):
            step(i % n_streams, streams[i % n_streams])
        torch.cuda.synchronize()
        # timed region: K steps issued back to back, alternating between the
        # streams, synchronised on both sides, with no events between the
        # kernels (an event record costs several microseconds of device time
        # per kernel boundary)
        t0 = time.perf_counter()
        for i in range(steps):
            step(i % n_streams, streams[i % n_streams])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        # the same K steps on one stream, no events: the single-stream rate
        t0 = time.perf_counter()
        for i in range(steps):
            step()
        torch.cuda.synchronize()
        wall1 = (time.perf_counter() - t0) * 1e3 / steps
        # and again on one stream with HIP events around every kernel on the
        # launch stream: per-kernel durations and per-step device latency
        for i in range(steps):
            step(ev=evs[i])
        torch.cuda.synchronize()
        stage_ms = {nm: [e[j].elapsed_time(e[j + 1]) for e in evs] for j, nm in enumerate(names)}
        total_ms = [e[0].elapsed_time(e[-1]) for e in evs]
        outs = [b[2] for b in bufs]
        for o in outs[1:]:
            if not torch.equal(o, outs[0]):
                raise RuntimeError("the streams' outputs differ")
        return outs[0], stage_ms, total_ms, wall, wall1

    # ---------------------------------------------------------- timed region
    log(f"timing mixed path ({'fused' if fuses['mixed'] else 'stack'}) ...")
    out_m, st_m, tot_m, wall_m, wall1_m = time_path("mixed", args.steps, args.warmup, fuses["mixed"])
    log(f"timing fp64 path ({'fused' if fuses['fp64'] else 'stack'}) ...")
    out_d, st_d, tot_d, wall_d, wall1_d = time_path("fp64", args.steps, args.warmup, fuses["fp64"])
    log("timing the other path of each precision ...")
    fu_steps = max(5, args.steps // 5)
    out_s, st_s, tot_s, wall_s, _ = time_path("mixed", fu_steps, 2, not fuses["mixed"])
    out_sd, st_sd, tot_sd, wall_sd, _ = time_path("fp64", fu_steps, 2, not fuses["fp64"])
    other_equal = bool(torch.equal(out_s, out_m) and torch.equal(out_sd, out_d))

    med = lambda v: float(np.median(v))
    # whole-job rate: K steps over the synchronised wall clock of the timed region
    ms_m, ms_d = wall_m, wall_d
    mpix = H * W / 1e6
    value = mpix / (ms_m * 1e-3)
    value_d = mpix / (ms_d * 1e-3)

    # brute force on the GPU (context)
    log("timing GPU brute force ...")
    bsteps = 3
    ob = abf.bruteforce(fd, sd, theta=td, kernel=kernel, rho=R, sigma_s=ss, precision="fp64")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(bsteps):
        abf.bruteforce(fd, sd, theta=td, kernel=kernel, rho=R, sigma_s=ss, precision="fp64", out=ob)
    e1.record()
    torch.cuda.synchronize()
    brute_ms = e0.elapsed_time(e1) / bsteps

    # ---------------------------------------------------------- roofline
    model = stage_model(H, W, kernel, R, N, 4, th is not None)
    stages = {k: med(v) for k, v in st_m.items()}
    dom = max(stages, key=stages.get)
    dur_s = stages[dom] * 1e-3
    gbs = model[dom]["bytes"] / dur_s / 1e9
    tfl = model[dom]["flops"] / dur_s / 1e12
    frac_h = gbs / HBM_PEAK_GBS
    frac_a = tfl / FP64_PEAK_TFLOPS
    if frac_a > frac_h:
        roof = {"bound": "alu", "achieved": round(tfl, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(frac_a, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(frac_h, 4)}
    roof.update({"kernel": dom, "traffic": measured_traffic(args.workload, dom),
                 "launch_ms": round(stages[dom], 5),
                 "algorithmic_bytes": model[dom]["bytes"], "algorithmic_flops": model[dom]["flops"]})

    # ---------------------------------------------------------- parity (CPU legs' oracle values)
    err_m = err_d = None
    n_par = 0
    if par_ref is not None:
        ys, xs = par_px
        err_m = float(np.max(np.abs(out_m.cpu().numpy().astype(np.float64)[ys, xs] - par_ref)))
        err_d = float(np.max(np.abs(out_d.cpu().numpy()[ys, xs] - par_ref)))
        n_par = int(len(ys))
    # whole path at the roofline: the algorithmic bytes of one step (read f,
    # theta-or-f and sigma, write the output, write and read once each plane
    # the path keeps in HBM: the whole stack, or on the fused path the window
    # bounds only; where one kernel runs the whole filter the bounds are
    # written and never read back) over the step's wall time
    planes = 2 if fuses["mixed"] else N + 2
    bpp = 16 + 8 * planes - (8 if fuses["mixed"] and single else 0)
    path_bytes = H * W * bpp
    path_gbs = path_bytes / (ms_m * 1e-3) / 1e9
    whole = {"bound": "hbm", "achieved": round(path_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(path_gbs / HBM_PEAK_GBS, 4), "bytes_per_step": path_bytes,
             "bytes_per_pixel": bpp}
    if fuses["mixed"]:
        # the same rate against the stack formulation's algorithmic bytes (the
        # whole moment stack written and read once): what the fused path
        # keeps out of HBM, expressed as a fraction of the HBM roofline
        sb = 16 + 8 * (N + 2)
        whole["stack_formulation_bytes_per_pixel"] = sb
        whole["frac_at_stack_formulation_bytes"] = round(H * W * sb / (ms_m * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    lat_m = np.array(tot_m)
    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_m, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "h": H, "w": W, "kernel": kernel, "rho": R, "N": N,
                   "sigma_s": ss, "precision": "mixed (FP64 arithmetic, FP32 stack and output)",
                   "streams": n_streams},
        "single_stream": {"value": round(mpix / (wall1_m * 1e-3), 2), "ms_per_step": round(wall1_m, 5),
                          "fp64_value": round(mpix / (wall1_d * 1e-3), 2)},
        "latency_ms": {"p50": round(float(np.percentile(lat_m, 50)), 5),
                       "p99": round(float(np.percentile(lat_m, 99)), 5)},
        "stage_ms_mixed": {k: round(v, 5) for k, v in stages.items()},
        "fp64": {"value": round(value_d, 2), "ms_per_step": round(ms_d, 5),
                 "stage_ms": {k: round(med(v), 5) for k, v in st_d.items()},
                 "max_abs_err_vs_oracle": err_d},
        "mixed_max_abs_err_vs_oracle": err_m,
        "parity_pixels": n_par,
        "brute_force_fp64": {"value": round(mpix / (brute_ms * 1e-3), 3), "ms": round(brute_ms, 3)},
        "device_ms_per_step_median": {"mixed": round(med(tot_m), 5), "fp64": round(med(tot_d), 5)},
        "path": {p: "fused" if f else "stack" for p, f in fuses.items()},
        "other_path": {"path": {p: "stack" if f else "fused" for p, f in fuses.items()},
                       "mixed_ms_per_step": round(wall_s, 5), "fp64_ms_per_step": round(wall_sd, 5),
                       "mixed_value": round(mpix / (wall_s * 1e-3), 2),
                       "stage_ms_mixed": {k: round(med(v), 5) for k, v in st_s.items()},
                       "stage_ms_fp64": {k: round(med(v), 5) for k, v in st_sd.items()},
                       "output_equals_path": other_equal},
        "roofline": roof,
        "whole_path_roofline": whole,
        "prewarm_steps": PREWARM_STEPS,
        "cpu_baseline": cpu,
    }
    if args.serving_requests > 0:
        from paper_1811_02308_amd.serve import bench as serve_bench
        log("serving stream ...")
        res["serving"] = serve_bench(n=args.serving_requests, warm=max(10, args.serving_requests // 10))
        res["serving"]["config"] = ("Poisson stream of mixed requests (sides 256-2048, 1:1 or 4:3, "
                                    "rho 3/5/10/20, N 5/6/8, box or Gaussian), mixed precision, "
                                    "4 slots, 16 GB budget, host copies included")
    print(json.dumps(res), flush=True)


def precision_table(args):
    """The precision sweep on the 4096 x 4096 Voronoi workload: box kernel,
    rho in {5, 20}, N = 5..8, mixed and FP64 paths on one stream. Per
    configuration: the median event-timed time of a whole fast-filter call
    (both paths), the largest |mixed - FP64| over every pixel, and both
    paths' largest error against the CPU oracle on sampled pixels (corners,
    edge midpoints and random pixels)."""
    import numpy as np
    import torch

    import oracle
    import paper_1811_02308_amd as abf
    from synth import workload

    torch.cuda.set_device(0)
    abf.lib()
    rows = []
    npx = 1500
    for R in (5, 20):
        for N in (5, 6, 7, 8):
            wl = workload(f"voronoi4096_box{R}_n{N}")
            f, sg = wl["f"], wl["sigma"]
            H, W = f.shape
            fd, sd = torch.from_numpy(f).cuda(), torch.from_numpy(sg).cuda()
            outs, ms = {}, {}
            for prec in ("mixed", "fp64"):
                ws = torch.empty(abf.workspace_bytes(H, W, R, N, prec), dtype=torch.uint8, device="cuda")
                out = torch.empty((H, W), dtype=torch.float32 if prec == "mixed" else torch.float64,
                                  device="cuda")
                call = lambda: abf.fast(fd, sd, kernel="box", rho=R, N=N, precision=prec, out=out,
                                        workspace=ws)
                for _ in range(PREWARM_STEPS // 3):
                    call()
                torch.cuda.synchronize()
                ts = []
                for _ in range(max(5, min(args.steps, 30))):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    call()
                    e1.record()
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1))
                ms[prec] = float(np.median(ts))
                outs[prec] = out.double().cpu().numpy()
            rng = np.random.default_rng(11 + R + N)
            ys = np.concatenate([[0, 0, H - 1, H - 1, H // 2, 0, H - 1, H // 2],
                                 rng.integers(0, H, npx)])
            xs = np.concatenate([[0, W - 1, 0, W - 1, 0, W // 2, W // 2, W - 1],
                                 rng.integers(0, W, npx)])
            ref = oracle.fast_abf(f, None, sg, "box", R, N, pixels=(ys, xs))
            row = {"rho": R, "N": N,
                   "mixed_ms": round(ms["mixed"], 4), "fp64_ms": round(ms["fp64"], 4),
                   "mixed_mpix_s": round(H * W / 1e3 / ms["mixed"], 1),
                   "fp64_mpix_s": round(H * W / 1e3 / ms["fp64"], 1),
                   "max_abs_mixed_minus_fp64_all_pixels": float(np.max(np.abs(outs["mixed"] - outs["fp64"]))),
                   "mixed_max_abs_err_vs_oracle": float(np.max(np.abs(outs["mixed"][ys, xs] - ref))),
                   "fp64_max_abs_err_vs_oracle": float(np.max(np.abs(outs["fp64"][ys, xs] - ref))),
                   "oracle_pixels": int(len(ys))}
            log(row)
            rows.append(row)
    print(json.dumps({"metric": "precision sweep, mixed vs FP64 error per N",
                      "config": {"workload": "voronoi4096 box rho 5/20, N 5..8 (one fast-filter call, one stream)"},
                      "rows": rows}), flush=True)


def kernel_sweep(args):
    """Where the recursive spatial kernel (cost independent of rho) would
    overtake the Gaussian tile kernel (cost linear in rho per axis): a
    4096 x 4096 smooth Gaussian field, N = 6, mixed path, one stream, rho in
    {8, 15, 25, 40, 60, 96}. Per rho: the median event-timed moment-stack
    call of each kernel and of the whole fast filter, the largest
    |recursive - Gaussian| output difference over every pixel (the two
    kernels' weights differ by Deriche's approximation error), and the
    recursive output's largest error against the CPU oracle on sampled
    pixels."""
    import numpy as np
    import torch

    import oracle
    import paper_1811_02308_amd as abf
    from synth import gauss_field, smooth_field

    torch.cuda.set_device(0)
    abf.lib()
    H = W = 4096
    N = 6
    f = gauss_field(1002, H, W)
    sg = smooth_field(np.random.default_rng(1), H, W, 5, 60)
    fd, sd = torch.from_numpy(f).cuda(), torch.from_numpy(sg).cuda()
    reps = max(5, min(args.steps, 10))

    def timed(call):
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            call()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    rng = np.random.default_rng(5)
    ys = np.concatenate([[0, 0, H - 1, H - 1], rng.integers(0, H, 60)])
    xs = np.concatenate([[0, W - 1, 0, W - 1], rng.integers(0, W, 60)])
    rows = []
    for R in (8, 15, 25, 40, 60, 96):
        row = {"rho": R, "N": N}
        outs = {}
        for kern in ("gaussian", "recursive"):
            st = torch.empty(abf.stack_bytes(H, W, N, "mixed"), dtype=torch.uint8, device="cuda")
            ws = torch.empty(abf.lib().abf_kernel_scratch_bytes(H, W, R, N, abf.KERNELS[kern]),
                             dtype=torch.uint8, device="cuda")
            wsf = torch.empty(abf.workspace_bytes(H, W, R, N, "mixed", kernel=kern), dtype=torch.uint8,
                              device="cuda")
            out = torch.empty((H, W), dtype=torch.float32, device="cuda")
            row[f"{kern}_stack_ms"] = round(timed(lambda: abf.moment_stack(
                fd, kernel=kern, rho=R, N=N, precision="mixed", stack=st, workspace=ws)), 4)
            row[f"{kern}_fast_ms"] = round(timed(lambda: abf.fast(
                fd, sd, kernel=kern, rho=R, N=N, precision="mixed", out=out, workspace=wsf)), 4)
            outs[kern] = out.double().cpu().numpy()
        row["max_abs_recursive_minus_gaussian"] = float(np.max(np.abs(outs["recursive"] - outs["gaussian"])))
        ref = oracle.fast_abf(f, None, sg, "recursive", R, N, pixels=(ys, xs))
        row["recursive_max_abs_err_vs_oracle"] = float(np.max(np.abs(outs["recursive"][ys, xs] - ref)))
        row["oracle_pixels"] = int(len(ys))
        log(row)
        rows.append(row)
    print(json.dumps({"metric": "moment-stack ms, Gaussian tile vs recursive kernel",
                      "config": {"workload": "gauss_field 4096x4096, N 6, mixed, rho 8..96 (one stream)"},
                      "rows": rows}), flush=True)


def batched_bench(args):
    """abf_fast_batched against a host loop of abf_fast calls over the same
    requests (each request in its own allocations, workspace and request
    table built once, both through the C ABI on one stream, mixed path):
    64 images of 256 x 256 (one group), a mix of 48 requests of three sizes
    and two parameter sets (six groups), and the 96 planes of 1920 x 1080 of
    the texture batch (one group; abf_fast_strided beside it). Per case: the
    median event-timed device time per call of each route and the outputs'
    equality."""
    import ctypes

    import numpy as np
    import torch

    import paper_1811_02308_amd as abf
    from synth import rect_scene, smooth_field

    torch.cuda.set_device(0)
    L = abf.lib()
    prec = 1
    reps = max(5, min(args.steps, 20))

    def timed(call):
        for _ in range(5):
            call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            call()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    scenes = {}

    def case(name, specs):
        reqs = (abf.Request * len(specs))()
        keep, outs_b, outs_l, singles = [], [], [], []
        for i, (h, w, kernel, R, N) in enumerate(specs):
            key = (i % 8, h, w)
            if key not in scenes:
                scenes[key] = (rect_scene(900 + i % 8, h, w, n_rect=6, noise=8.0, side_lo=4,
                                          side_hi=max(5, min(h, w) // 2)),
                               smooth_field(np.random.default_rng(i % 8), h, w, 8, 40))
            f = torch.from_numpy(scenes[key][0]).cuda()
            sg = torch.from_numpy(scenes[key][1]).cuda()
            ob = torch.empty((h, w), dtype=torch.float32, device="cuda")
            ol = torch.empty_like(ob)
            ws = torch.empty(abf.workspace_bytes(h, w, R, N, "mixed", kernel=kernel), dtype=torch.uint8,
                             device="cuda")
            keep += [f, sg, ws]
            outs_b.append(ob)
            outs_l.append(ol)
            reqs[i] = abf.Request(f.data_ptr(), None, sg.data_ptr(), h, w, w, abf.KERNELS[kernel], 0.0,
                                  R, N, ob.data_ptr(), w)
            singles.append((ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(sg.data_ptr()), h, w,
                            abf.KERNELS[kernel], R, N, ctypes.c_void_p(ol.data_ptr()),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        n = len(specs)
        wsb = L.abf_batched_workspace_bytes(reqs, n, prec)
        bws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

        def batched():
            st = L.abf_fast_batched(reqs, n, prec, abf.FLAG_CLAMP, ctypes.c_void_p(bws.data_ptr()), wsb,
                                    stream)
            if st != 0:
                raise RuntimeError(f"abf_fast_batched: {st}")

        def loop():
            for (fp, sp, h, w, kind, R, N, op, wp, wn) in singles:
                st = L.abf_fast(fp, None, sp, h, w, w, kind, 0.0, R, N, prec, abf.FLAG_CLAMP, op, w, wp,
                                wn, stream)
                if st != 0:
                    raise RuntimeError(f"abf_fast: {st}")

        row = {"case": name, "requests": n, "groups": len({s for s in specs}),
               "mpix": round(sum(h * w for h, w, *_ in specs) / 1e6, 3)}
        row["loop_ms"] = round(timed(loop), 4)
        row["batched_ms"] = round(timed(batched), 4)
        row["loop_mpix_s"] = round(row["mpix"] * 1e3 / row["loop_ms"], 1)
        row["batched_mpix_s"] = round(row["mpix"] * 1e3 / row["batched_ms"], 1)
        row["speedup"] = round(row["loop_ms"] / row["batched_ms"], 3)
        torch.cuda.synchronize()
        row["outputs_equal"] = all(torch.equal(a, b) for a, b in zip(outs_b, outs_l))
        if name == "texture_planes":
            h, w, kernel, R, N = specs[0]
            x = torch.stack([keep[3 * i] for i in range(n)])
            sgs = torch.stack([keep[3 * i + 1] for i in range(n)])
            out = torch.empty_like(x)
            sws = torch.empty(L.abf_strided_workspace_bytes(n, h, w, R, N, prec), dtype=torch.uint8,
                              device="cuda")
            row["strided_ms"] = round(timed(lambda: abf.fast_strided(
                x, sgs, kernel=kernel, rho=R, N=N, precision="mixed", out=out, workspace=sws)), 4)
        log(row)
        return row

    rows = [case("small_256", [(256, 256, "box", 5, 6)] * 64)]
    mix = []
    for i in range(48):
        side = (256, 512, 1024)[i % 3]
        mix.append((side, side, "box", 5, 6) if i % 2 else (side, side * 4 // 3, "gaussian", 3, 5))
    rows.append(case("mixed_sizes", mix))
    rows.append(case("texture_planes", [(1080, 1920, "box", 8, 6)] * 96))
    print(json.dumps({"metric": "ms per batch, abf_fast_batched vs a loop of abf_fast",
                      "config": {"workload": "batches of independent requests, mixed path, one stream"},
                      "rows": rows}), flush=True)


def classical_bench(args):
    """Classical filter (theta = f, sigma = 40) on the 512 x 512 scene of
    Sec. III-B's sweeps: GPU time of the fast path for rho in {3..11} and
    N in {1, 3, 5} next to the GPU brute force (the structure of the paper's
    timing table), and the PSNR against brute force for rho in {3, 5, 10},
    N = 0..6, with the uniform-prior variant beside N = 0."""
    import numpy as np
    import torch

    import paper_1811_02308_amd as abf
    from synth import workload
    wl = workload("classical512_box5_n5")
    f = wl["f"]
    H, W = f.shape
    img = torch.from_numpy(f).cuda()
    sg = torch.from_numpy(wl["sigma"]).cuda()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(5, min(args.steps, 50))
    timing = {}
    for R in (3, 5, 7, 9, 11):
        row = {}
        for N in (1, 3, 5):
            for prec in ("mixed", "fp64"):
                ws = torch.empty(abf.workspace_bytes(H, W, R, N, prec), dtype=torch.uint8, device="cuda")
                out = torch.empty((H, W), dtype=torch.float32 if prec == "mixed" else torch.float64,
                                  device="cuda")
                row[f"N={N} {prec} ms"] = round(timed(
                    lambda: abf.fast(img, sg, kernel="box", rho=R, N=N, precision=prec, out=out,
                                     workspace=ws), reps), 5)
        ob = torch.empty((H, W), dtype=torch.float64, device="cuda")
        row["brute fp64 ms"] = round(timed(
            lambda: abf.bruteforce(img, sg, kernel="box", rho=R, precision="fp64", out=ob), 3), 4)
        timing[f"rho={R}"] = row
        log(f"rho={R}: {row}")
    psnr = {}
    for R in (3, 5, 10):
        b = abf.bruteforce(img, sg, kernel="box", rho=R, precision="fp64").cpu().numpy()
        p = lambda g: round(float(10 * np.log10(255.0 ** 2 / np.mean(
            (g.cpu().numpy().astype(np.float64) - b) ** 2))), 2)
        psnr[f"rho={R}"] = {
            "fp64": [p(abf.fast(img, sg, kernel="box", rho=R, N=N, precision="fp64")) for N in range(7)],
            "mixed": [p(abf.fast(img, sg, kernel="box", rho=R, N=N, precision="mixed")) for N in range(7)],
            "uniform_prior": p(abf.uniform_prior(img, sg, kernel="box", rho=R, precision="fp64")),
        }
        log(f"rho={R}: PSNR {psnr[f'rho={R}']}")
    res = {"metric": "classical-filter sweep (theta = f, sigma = 40, box kernel)",
           "config": {"workload": "classical512_box5_n5", "h": H, "w": W},
           "timing_ms": timing, "psnr_db_vs_bruteforce": psnr,
           "notes": "PSNR lists are N = 0..6; uniform_prior is the N = 0 estimator on [f, 2 fbar - f]"}
    print(json.dumps(res), flush=True)


def paper_maps_bench(args):
    """The applications of Sec. IV with the paper's own parameter maps, all
    on the GPU: sharpening of the 1024 x 1024 field (theta = 2 f - fbar over
    the 31 x 31 window, sigma from |LoG|; Gaussian kernel R = 15, N = 6) and
    the three-pass texture procedure (mRTV sigma, 0.8 sigma, sharpening) on
    the 32 RGB 1920 x 1080 frames (box R = 8, N = 6)."""
    import numpy as np
    import torch

    import paper_1811_02308_amd as abf
    from synth import workload

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(reps):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / reps, (time.perf_counter() - t0) * 1e3 / reps

    res = {"metric": "applications with the paper's parameter maps (Sec. IV)"}
    sw = workload("sharpen1024_gauss15_n6")
    f = torch.from_numpy(sw["f"]).cuda()
    H, W = f.shape
    ws = torch.empty(abf.workspace_bytes(H, W, 15, 6, "mixed"), dtype=torch.uint8, device="cuda")
    out = torch.empty((H, W), dtype=torch.float32, device="cuda")

    def sharpen():
        th, sg = abf.sharpen_maps(f, radius=15, log_sigma=1.0, lo=5.0, hi=40.0, v_ref=20.0)
        return abf.fast(f, sg[0], theta=th[0], kernel="gaussian", rho=15, N=6, sigma_s=5.0,
                        out=out, workspace=ws), th, sg
    (_, th, sg), dev_ms, wall_ms = timed(sharpen, max(5, min(args.steps, 50)))
    res["sharpening"] = {
        "workload": "sharpen1024 field, maps from the image, Gaussian R=15 N=6, mixed",
        "ms_per_image": round(wall_ms, 4), "device_ms": round(dev_ms, 4),
        "mpix_per_s": round(H * W / 1e6 / (wall_ms * 1e-3), 1),
        "max_abs_err_vs_oracle": None, "maps_max_abs_err_vs_oracle_200x200": None}
    if not args.no_cpu_baseline:
        # cpu_baseline leg: the CPU oracle (one thread) on 300 random pixels
        # of the filter fed the GPU's maps, and the maps on a 200 x 200 crop;
        # the same values give the parity
        import oracle
        from oracle import maps
        rng = np.random.default_rng(3)
        ys, xs = rng.integers(0, H, 300), rng.integers(0, W, 300)
        with one_host_thread():
            t0 = time.perf_counter()
            ref = oracle.fast_abf(sw["f"], th[0].cpu().numpy(), sg[0].cpu().numpy(), "gaussian", 15,
                                  6, sigma_s=5.0, pixels=(ys, xs))
            dt = time.perf_counter() - t0
            rth, rsg = maps.sharpen_maps(sw["f"][:200, :200], 15, 1.0, 5.0, 40.0, 20.0)
        res["sharpening"]["max_abs_err_vs_oracle"] = float(
            np.max(np.abs(out.cpu().numpy().astype(np.float64)[ys, xs] - ref)))
        res["sharpening"]["maps_max_abs_err_vs_oracle_200x200"] = float(max(
            np.max(np.abs(th[0].cpu().numpy()[:200, :200] - rth)[20:-20, 20:-20]),
            np.max(np.abs(sg[0].cpu().numpy()[:200, :200] - rsg)[20:-20, 20:-20])))
        res["cpu_baseline"] = {"value": round(len(ys) / dt / 1e6, 6), "unit": "Mpix/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{len(ys)} random pixels of the sharpening filter, 1 thread, "
                                         f"{dt:.1f} s"}
    log("sharpening:", res["sharpening"])
    tw = workload("texture1080_box8_n6")
    n3, h, w = tw["frames"].shape
    fr = torch.from_numpy(tw["frames"]).cuda().view(n3 // 3, 3, h, w)
    for prec in ("mixed", "fp64"):
        _, dev_ms, wall_ms = timed(lambda: abf.texture_filter_paper(fr, rho=8, N=6, precision=prec), 2)
        res[f"texture_{prec}"] = {"ms_per_call": round(wall_ms, 3), "device_ms": round(dev_ms, 3),
                                  "mpix_per_s": round(3 * n3 * h * w / 1e6 / (wall_ms * 1e-3), 1)}
        log(f"texture {prec}:", res[f"texture_{prec}"])
    res["config"] = {"texture": "32 RGB 1920x1080 frames, box R=8 N=6, 3 passes (mRTV sigma, 0.8 sigma, sharpening)"}
    print(json.dumps(res), flush=True)


def texture_bench(args):
    """Texture workload: 32 RGB frames as 96 planes, 3 passes of
    (sigma map, batched fast filter), one launch per stage per pass."""
    import numpy as np
    import torch

    import paper_1811_02308_amd as abf
    from synth import workload
    wl = workload(args.workload)
    frames = wl["frames"]
    n, H, W = frames.shape
    R, N, passes = wl["R"], wl["N"], wl["passes"]
    sr = wl["sigma_rule"]
    log(f"texture workload: {n} planes of {H}x{W}, box R={R}, N={N}, {passes} passes")
    x = torch.from_numpy(frames).cuda()

    def run(prec, steps, warmup):
        for _ in range(warmup):
            abf.texture_filter(x, passes, R, N, precision=prec, **sr)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            out = abf.texture_filter(x, passes, R, N, precision=prec, **sr)
        e1.record()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3 / steps, e0.elapsed_time(e1) / steps

    steps = max(1, min(args.steps, 5))
    out_m, ms_m, dev_m = run("mixed", steps, 1)
    out_d, ms_d, dev_d = run("fp64", steps, 1)
    mpix = passes * n * H * W / 1e6
    # cpu_baseline leg: the CPU oracle (one thread) on sampled pixels of the
    # last pass of three planes, fed the GPU's own pass input and sigma map;
    # the same values give the parity
    errs = {"mixed": None, "fp64": None}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(5)
        npx, tsum = 0, 0.0
        for prec in ("mixed", "fp64"):
            prev = abf.texture_filter(x, passes - 1, R, N, precision=prec, **sr).float() if passes > 1 else x
            sig = abf.sigma_local_std(prev, **sr)
            last = abf.fast_strided(prev, sig, kernel="box", rho=R, N=N, precision=prec)
            errs[prec] = 0.0
            for c in (0, n // 2, n - 1):
                ys, xs = rng.integers(0, H, 150), rng.integers(0, W, 150)
                pc, sc = prev[c].cpu().numpy(), sig[c].cpu().numpy()
                with one_host_thread():
                    t0 = time.perf_counter()
                    ref = oracle.fast_abf(pc, None, sc, "box", R, N, pixels=(ys, xs))
                    tsum += time.perf_counter() - t0
                npx += len(ys)
                got = last[c].cpu().numpy().astype(np.float64)[ys, xs]
                errs[prec] = max(errs[prec], float(np.max(np.abs(got - ref))))
        cpu = {"value": round(npx / tsum / 1e6, 6), "unit": "Mpix/s", "cores": 1, "kind": "oracle",
               "sample": f"{npx} random pixels of the last pass (3 planes, both precisions' inputs), "
                         f"1 thread, {tsum:.1f} s"}
    res = {"metric": METRIC, "value": round(mpix / (ms_m * 1e-3), 2), "unit": "Mpix/s", "n_gpus": 1,
           "steps": steps, "warmup": 1, "ms_per_step": round(ms_m, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": args.workload, "planes": n, "h": H, "w": W, "kernel": "box", "rho": R,
                      "N": N, "passes": passes, "precision": "mixed (FP64 arithmetic, FP32 stack and output)"},
           "device_ms_per_step": round(dev_m, 4),
           "fp64": {"value": round(mpix / (ms_d * 1e-3), 2), "ms_per_step": round(ms_d, 4),
                    "max_abs_err_vs_oracle": errs["fp64"]},
           "mixed_max_abs_err_vs_oracle": errs["mixed"], "roofline": None, "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
