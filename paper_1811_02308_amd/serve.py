"""Continuous-batching request loop for the fast adaptive bilateral filter.

Requests (an image id with its pixels, a sigma map, optional theta, and the
filter parameters) arrive over time. One host thread runs the loop:

  * arrivals enter a FIFO queue;
  * the head request is admitted when a slot (a HIP stream) is free and its
    device footprint fits the free part of the memory budget; requests keep
    arriving and being admitted while others run, so the device works on
    several requests at once, each on its own stream;
  * admission enqueues everything a request needs on its slot's stream:
    upload of what is not resident, the filter (abf_fast, or only abf_range
    when the moment stack of the same image, kernel, rho and N is resident),
    the download of the result, and an event;
  * completed events free the slot and the request's transient memory; the
    result and its latency (completion - arrival) are recorded.

Images, sigma maps that carry an identity (``sigma_id``) and moment stacks
are kept resident in HBM in LRU caches whose bytes count against the same
budget (the stack depends only on the image, kernel, rho and N, so a request
that changes only theta or sigma reuses it; a request whose image and sigma
map are resident moves only its result over PCIe).

The device work goes through an *executor*. ``GPUExecutor`` drives the HIP
library; ``FakeExecutor`` (tests) runs on the CPU with modelled durations, so
admission, memory accounting, ordering and failure handling are testable
without a GPU. A request whose launch raises is marked failed and the loop
goes on.
"""
from __future__ import annotations

import collections
import dataclasses
import json
import math
import sys
import time
from typing import Any, Dict, List, Optional


@dataclasses.dataclass
class Request:
    id: int
    t_arrival: float                     # seconds from the start of the run
    image_id: Any                        # identity of the pixels (cache key)
    f: Any                               # host float32 (h, w)
    sigma: Any                           # host float32 (h, w)
    theta: Any = None
    kernel: str = "box"
    sigma_id: Any = None                 # identity of the sigma map (cache key); None: upload
    sigma_s: float = 0.0
    rho: int = 3
    N: int = 5

    @property
    def shape(self):
        return self.f.shape

    @property
    def pixels(self) -> int:
        return int(self.f.shape[0] * self.f.shape[1])


@dataclasses.dataclass
class Result:
    id: int
    t_arrival: float
    t_admit: float
    t_done: float
    ok: bool
    out: Any = None
    error: str = ""
    stack_hit: bool = False

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class LRUBytes:
    """An LRU cache with a byte budget. Entries in use by an in-flight
    request are held (reference count) and never evicted."""

    def __init__(self):
        self.d: "collections.OrderedDict[Any, list]" = collections.OrderedDict()
        self.bytes = 0

    def get(self, key):
        v = self.d.get(key)
        if v is not None:
            self.d.move_to_end(key)
            return v[0]
        return None

    def put(self, key, value, nbytes):
        if key in self.d:
            old = self.d.pop(key)
            self.bytes -= old[1]
        self.d[key] = [value, nbytes, 0]
        self.bytes += nbytes

    def hold(self, key):
        if key in self.d:
            self.d[key][2] += 1

    def unhold(self, key):
        if key in self.d:
            self.d[key][2] -= 1

    def evict_one(self):
        for k, v in self.d.items():
            if v[2] == 0:
                self.bytes -= v[1]
                del self.d[k]
                return True
        return False


class Server:
    def __init__(self, executor, mem_budget: int, poll_s: float = 5e-5):
        self.ex = executor
        self.budget = int(mem_budget)
        self.poll_s = poll_s
        self.images = LRUBytes()
        self.maps = LRUBytes()
        self.stacks = LRUBytes()
        self.transient = 0
        self.max_in_use = 0

    # ------------------------------------------------------------------ memory
    def in_use(self) -> int:
        return self.transient + self.images.bytes + self.maps.bytes + self.stacks.bytes

    def _make_room(self, need: int) -> bool:
        while self.in_use() + need > self.budget:
            if not (self.stacks.evict_one() or self.maps.evict_one() or self.images.evict_one()):
                return False
        return True

    # ------------------------------------------------------------------ loop
    def run(self, requests: List[Request], realtime: bool = True,
            timeout_s: float = 600.0) -> List[Result]:
        """Serve ``requests`` (arrival times in seconds from the start).
        realtime=False runs on the executor's virtual clock (tests)."""
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        queue: "collections.deque[Request]" = collections.deque()
        inflight: List[tuple] = []
        results: Dict[int, Result] = {}
        i = 0
        t0 = time.perf_counter()
        vt = 0.0
        now_fn = (lambda: time.perf_counter() - t0) if realtime else (lambda: vt)
        while len(results) < len(reqs):
            now = now_fn()
            if realtime and now > timeout_s:
                raise TimeoutError("serving loop exceeded its time limit")
            if not realtime:
                self.ex.now = vt
            while i < len(reqs) and reqs[i].t_arrival <= now:
                queue.append(reqs[i])
                i += 1
            # completions
            still = []
            for (r, h, t_adm, nbytes, hit, keys) in inflight:
                if self.ex.done(h):
                    t_done = now_fn() if realtime else self.ex.finish_time(h)
                    try:
                        out = self.ex.result(h)
                        results[r.id] = Result(r.id, r.t_arrival, t_adm, t_done, True, out,
                                               stack_hit=hit)
                    except Exception as e:                 # failure surfaced at completion
                        results[r.id] = Result(r.id, r.t_arrival, t_adm, t_done, False,
                                               error=repr(e))
                    self.ex.release(h)
                    self.transient -= nbytes
                    self.images.unhold(keys[0])
                    self.maps.unhold(keys[1])
                    self.stacks.unhold(keys[2])
                else:
                    still.append((r, h, t_adm, nbytes, hit, keys))
            inflight = still
            # admissions: FIFO, the head waits for room rather than being overtaken
            while queue and len(inflight) < self.ex.n_slots:
                r = queue[0]
                skey = (r.image_id, r.kernel, r.rho, r.N, r.sigma_s)
                mkey = r.sigma_id
                have_img = self.images.get(r.image_id) is not None
                have_map = mkey is not None and self.maps.get(mkey) is not None
                have_stack = self.stacks.get(skey) is not None
                img_b, map_b, stack_b, tmp_b = self.ex.footprint(r)
                need = (tmp_b + (0 if have_img else img_b) + (0 if have_map else map_b) +
                        (0 if have_stack else stack_b))
                if tmp_b + img_b + map_b + stack_b > self.budget:
                    queue.popleft()
                    results[r.id] = Result(r.id, r.t_arrival, now, now, False,
                                           error="request larger than the memory budget")
                    continue
                # hold what this request reuses so that making room cannot evict it
                self.images.hold(r.image_id)
                self.maps.hold(mkey)
                self.stacks.hold(skey)
                if not self._make_room(need):
                    self.images.unhold(r.image_id)
                    self.maps.unhold(mkey)
                    self.stacks.unhold(skey)
                    break
                t_adm = now_fn()
                try:
                    h, img_handle, map_handle, stack_handle = self.ex.launch(
                        r, self.images.get(r.image_id),
                        None if mkey is None else self.maps.get(mkey), self.stacks.get(skey), t_adm)
                except Exception as e:
                    self.images.unhold(r.image_id)
                    self.maps.unhold(mkey)
                    self.stacks.unhold(skey)
                    queue.popleft()
                    results[r.id] = Result(r.id, r.t_arrival, t_adm, t_adm, False, error=repr(e))
                    continue
                queue.popleft()
                if not have_img:
                    self.images.put(r.image_id, img_handle, img_b)
                    self.images.hold(r.image_id)
                if mkey is not None and not have_map:
                    self.maps.put(mkey, map_handle, map_b)
                    self.maps.hold(mkey)
                if not have_stack:
                    self.stacks.put(skey, stack_handle, stack_b)
                    self.stacks.hold(skey)
                self.transient += tmp_b
                self.max_in_use = max(self.max_in_use, self.in_use())
                inflight.append((r, h, t_adm, tmp_b, have_stack, (r.image_id, mkey, skey)))
            if realtime:
                if self.poll_s > 0:
                    time.sleep(self.poll_s)
            else:
                # virtual clock: jump to the next event (arrival or completion)
                nxt = [self.ex.finish_time(h) for (_, h, _, _, _, _) in inflight]
                if i < len(reqs):
                    nxt.append(reqs[i].t_arrival)
                if nxt:
                    vt = max(vt, min(nxt))
        return [results[r.id] for r in requests]


def summarize(results: List[Result], wall_s: Optional[float] = None) -> dict:
    ok = [r for r in results if r.ok]
    lat = sorted(r.latency for r in ok)

    def pct(p):
        if not lat:
            return None
        k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
        return lat[k]

    px = sum(int(r.out.shape[0] * r.out.shape[1]) for r in ok if r.out is not None)
    span = wall_s if wall_s is not None else (max(r.t_done for r in ok) - min(r.t_arrival for r in ok)) if ok else 0
    return {"requests": len(results), "ok": len(ok), "failed": len(results) - len(ok),
            "p50_ms": None if not lat else 1e3 * pct(50), "p99_ms": None if not lat else 1e3 * pct(99),
            "mpix_per_s": (px / span / 1e6) if span > 0 else None,
            "stack_hits": sum(1 for r in ok if r.stack_hit)}


# ---------------------------------------------------------------------- executors
class FakeExecutor:
    """CPU stand-in on a virtual clock: a request occupies one of ``n_slots``
    for a time proportional to its pixels (less when its stack is reused) and
    returns ``compute(r)`` (default: a copy of its image). ``fail_ids``
    raise at launch; ``fail_at_result`` raise when the result is fetched."""

    def __init__(self, n_slots=4, us_per_px=1e-3, fail_ids=(), fail_at_result=(), compute=None):
        self.n_slots = n_slots
        self.us_per_px = us_per_px
        self.fail_ids = set(fail_ids)
        self.fail_at_result = set(fail_at_result)
        self.compute = compute
        self.launched = []
        self.map_uploads = 0
        self.now = 0.0
        self._busy_until = [0.0] * n_slots
        self._slot_of = {}

    def footprint(self, r):
        """(image, sigma map when cached, stack, transient) bytes."""
        px = r.pixels
        cached = r.sigma_id is not None
        return (4 * px, 4 * px * cached, 4 * px * (r.N + 2),
                4 * px + 4 * px * (not cached) + 4 * px * (r.theta is not None))

    def launch(self, r, img_handle, map_handle, stack_handle, t_admit):
        if r.id in self.fail_ids:
            raise RuntimeError(f"injected failure for request {r.id}")
        free = [s for s in range(self.n_slots) if self._busy_until[s] <= t_admit]
        slot = free[0] if free else min(range(self.n_slots), key=lambda s: self._busy_until[s])
        start = max(t_admit, self._busy_until[slot])
        dur = r.pixels * self.us_per_px * 1e-6 * (0.3 if stack_handle is not None else 1.0)
        self._busy_until[slot] = start + dur
        self.launched.append(r.id)
        if r.sigma_id is not None and map_handle is None:
            self.map_uploads += 1
        return ({"r": r, "end": start + dur}, ("img", r.image_id),
                None if r.sigma_id is None else ("map", r.sigma_id), ("stack", r.image_id))

    def finish_time(self, h):
        return h["end"]

    def done(self, h):
        return h["end"] <= self.now

    def result(self, h):
        r = h["r"]
        if r.id in self.fail_at_result:
            raise RuntimeError(f"injected completion failure for request {r.id}")
        return self.compute(r) if self.compute else r.f.copy()

    def release(self, h):
        pass


class GPUExecutor:
    """Runs requests on the MI355X through the HIP library, one torch (HIP)
    stream per slot, default priority. Inputs are staged through pinned host
    memory; the result is copied back into pinned memory on the same stream
    and an event marks completion.

    Resident images and stacks are produced on one slot's stream and may be
    used by a request on another slot before that work has finished: every
    cached handle carries the event recorded after its producer's work, and
    a consumer's stream waits for it before using the handle. Theta is
    per request (it is not part of the cached image)."""

    def __init__(self, n_slots=4, precision="mixed", device=0, pinned_cap_bytes=2 << 30):
        import torch
        import paper_1811_02308_amd as abf
        self.torch, self.abf = torch, abf
        self.n_slots = n_slots
        self.precision = precision
        self.dev = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(n_slots)]
        # uploads of inputs that stay resident (images, sigma maps with an
        # identity) go on their own stream, so that a request on another slot
        # that reuses them waits for the copy only, not for the compute queued
        # on the uploading request's slot
        self.copy_stream = torch.cuda.Stream(device=self.dev)
        self.free_slots = list(range(n_slots))
        # pinned staging copies of host arrays reused across requests, LRU by
        # bytes (a dropped copy stays valid for copies already enqueued: torch's
        # pinned allocator keeps the block until they have run)
        self._pinned = collections.OrderedDict()   # id(host array) -> (pinned, array)
        self._pinned_bytes = 0
        self.pinned_cap = int(pinned_cap_bytes)
        abf.lib()

    def _pin(self, a):
        key = id(a)
        t = self._pinned.get(key)
        if t is not None and t[1] is a:
            self._pinned.move_to_end(key)
            return t[0]
        if t is not None:
            self._pinned_bytes -= t[0].numel() * t[0].element_size()
            del self._pinned[key]
        pin = self.torch.from_numpy(a).pin_memory()
        nb = pin.numel() * pin.element_size()
        while self._pinned and self._pinned_bytes + nb > self.pinned_cap:
            _, (old, _) = self._pinned.popitem(last=False)
            self._pinned_bytes -= old.numel() * old.element_size()
        self._pinned[key] = (pin, a)
        self._pinned_bytes += nb
        return pin

    def footprint(self, r):
        h, w = r.shape
        L = self.abf.lib()
        p = self.abf.PRECISIONS[self.precision]
        img_b = 4 * h * w
        cached = r.sigma_id is not None
        map_b = 4 * h * w * cached
        stack_b = int(L.abf_stack_bytes(h, w, r.N, p))
        ob = 4 if self.precision == "mixed" else 8
        tmp_b = (4 * h * w * ((not cached) + (r.theta is not None)) + ob * h * w +
                 int(L.abf_scratch_bytes(h, w, r.rho)))
        return img_b, map_b, stack_b, tmp_b

    def launch(self, r, img_handle, map_handle, stack_handle, t_admit):
        torch, abf = self.torch, self.abf
        slot = self.free_slots.pop(0)
        s = self.streams[slot]
        h, w = r.shape
        p = abf.PRECISIONS[self.precision]
        def resident_upload(a):
            with torch.cuda.stream(self.copy_stream):
                d = self._pin(a).to(self.dev, non_blocking=True)
                ev_up = torch.cuda.Event()
                ev_up.record(self.copy_stream)
            return d, ev_up

        if img_handle is None:
            img_handle = resident_upload(r.f)
        if map_handle is None and r.sigma_id is not None:
            map_handle = resident_upload(r.sigma)
        with torch.cuda.stream(s):
            s.wait_event(img_handle[1])
            fd = img_handle[0]
            td = None
            if r.theta is not None:
                td = self._pin(r.theta).to(self.dev, non_blocking=True)
            sp = None
            if map_handle is not None:
                s.wait_event(map_handle[1])
                sd = map_handle[0]
            else:
                sp = self._pin(r.sigma)
                sd = sp.to(self.dev, non_blocking=True)
            out = torch.empty((h, w), dtype=torch.float32 if p else torch.float64, device=self.dev)
            if stack_handle is None:
                stack = torch.empty(int(abf.lib().abf_stack_bytes(h, w, r.N, p)), dtype=torch.uint8,
                                    device=self.dev)
                abf.moment_stack(fd, kernel=r.kernel, rho=r.rho, N=r.N, sigma_s=r.sigma_s,
                                 precision=self.precision, stack=stack, stream=s)
                ev_stack = torch.cuda.Event()
                ev_stack.record(s)
                stack_handle = (stack, ev_stack)
            else:
                s.wait_event(stack_handle[1])
            abf.range_from_stack(stack_handle[0], sd, img=fd, theta=td, N=r.N,
                                 precision=self.precision, out=out, stream=s)
            host = torch.empty((h, w), dtype=out.dtype, pin_memory=True)
            host.copy_(out, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        # keep the transient tensors alive until the event has passed
        return ({"slot": slot, "ev": ev, "host": host, "keep": (sp, sd, td, out)}, img_handle,
                map_handle, stack_handle)

    def done(self, h):
        return h["ev"].query()

    def finish_time(self, h):
        raise NotImplementedError

    def result(self, h):
        return h["host"].numpy()

    def release(self, h):
        self.free_slots.append(h["slot"])
        h["keep"] = None


# ---------------------------------------------------------------------- benchmark
# Scenes and sigma maps of the request pool, keyed by (h, w, index): their
# seeds depend only on the key, so every stream draws from the same pool.
_SCENES: dict = {}
_SIGMAS: dict = {}


def make_requests(seed: int, n: int, rate: float, pool: int = 12, scale: float = 1.0):
    """Poisson arrivals of filter requests (sizes, rho, N, kernel as in the
    serving workload), drawing images from a pool of ``pool`` seeded scenes
    so that generation stays cheap; ``scale`` shrinks the side lengths."""
    import numpy as np
    from synth.generators import rect_scene, smooth_field
    rng = np.random.Generator(np.random.PCG64(seed))
    scenes = _SCENES
    sigmas = _SIGMAS
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        s = int(rng.choice([256, 512, 1024, 2048]) * scale)
        tall = bool(rng.random() < 0.5)
        h, w = (s, s) if tall else (s, int(round(4 * s / 3)))
        R = int(rng.choice([3, 5, 10, 20]))
        N = int(rng.choice([5, 6, 8]))
        gauss = bool(rng.random() < 0.5)
        k = int(rng.integers(0, pool))
        key = (h, w, k)
        if key not in scenes:
            f = rect_scene(10_000 + 97 * k + h, h, w, side_lo=max(1, h // 16), side_hi=max(2, h // 2))
            scenes[key] = f
        k2 = int(rng.integers(0, 4))
        if (h, w, k2) not in sigmas:
            sigmas[(h, w, k2)] = smooth_field(np.random.Generator(np.random.PCG64(7919 * k2 + h + w)),
                                              h, w, 10, 30)
        sig = sigmas[(h, w, k2)]
        out.append(Request(id=i, t_arrival=t, image_id=key, f=scenes[key], sigma=sig,
                           sigma_id=("sigma", h, w, k2),
                           kernel="gaussian" if gauss else "box",
                           sigma_s=R / 3.0 if gauss else 0.0, rho=R, N=N))
    return out


def breakdown(reqs, precision="mixed"):
    """Where the saturation rate goes: the same requests' filter calls alone
    (inputs resident, one stream, back to back), their host-device copies
    alone (image and sigma up, result down, pinned host memory: what a
    request moves when nothing it needs is resident), and the serving loop
    alone (a CPU executor that finishes every request at once)."""
    import torch
    import paper_1811_02308_amd as abf
    dev = torch.device("cuda")
    uniq = {}
    for r in reqs:
        uniq.setdefault(id(r.f), r.f)
        uniq.setdefault(id(r.sigma), r.sigma)
    resident = {k: torch.from_numpy(a).to(dev) for k, a in uniq.items()}
    pinned = {k: torch.from_numpy(a).pin_memory() for k, a in uniq.items()}
    px = sum(r.pixels for r in reqs)
    outs = {}
    for r in reqs:
        outs.setdefault(r.shape, torch.empty(r.shape, dtype=torch.float32 if precision == "mixed"
                                             else torch.float64, device=dev))

    def compute():
        for r in reqs:
            abf.fast(resident[id(r.f)], resident[id(r.sigma)], kernel=r.kernel, rho=r.rho, N=r.N,
                     sigma_s=r.sigma_s, precision=precision, out=outs[r.shape])

    def copies():
        for r in reqs:
            resident[id(r.f)].copy_(pinned[id(r.f)], non_blocking=True)
            resident[id(r.sigma)].copy_(pinned[id(r.sigma)], non_blocking=True)
            host = torch.empty(r.shape, dtype=outs[r.shape].dtype, pin_memory=True)
            host.copy_(outs[r.shape], non_blocking=True)

    res = {}
    for name, fn in (("compute_only", compute), ("copies_only", copies)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        res[name + "_mpix_per_s"] = px / (time.perf_counter() - t0) / 1e6
    loop_reqs = [dataclasses.replace(r, t_arrival=0.0) for r in reqs]
    ex = FakeExecutor(n_slots=4, us_per_px=0.0, compute=lambda r: None)
    t0 = time.perf_counter()
    Server(ex, 1 << 62, poll_s=0.0).run(loop_reqs, realtime=False)
    res["loop_only_req_per_s"] = len(reqs) / (time.perf_counter() - t0)
    res["requests"] = len(reqs)
    return res


def bench(loads=(0.3, 0.6, 0.9), n=300, warm=30, slots=4, budget_gb=16.0, seed=1004,
          precision="mixed", scale=1.0):
    """Measure closed-loop saturation throughput, then run Poisson streams at
    the given fractions of it; returns a dict with p50/p99 and Mpix/s per load.
    One executor serves every stream, as one server process would: its
    streams and pinned staging copies persist from run to run (the resident
    image and stack caches belong to each run's Server and start empty)."""
    import numpy as np
    ex = GPUExecutor(n_slots=slots, precision=precision)
    budget = int(budget_gb * (1 << 30))
    sat_reqs = make_requests(seed, n, 1e9, scale=scale)      # all arrive at once
    # one untimed pass of the same stream first: the executor's first uses of
    # the request pool's host arrays pin them, which a running server has done
    Server(ex, budget).run(sat_reqs)
    srv = Server(ex, budget)
    t0 = time.perf_counter()
    res = srv.run(sat_reqs)
    wall = time.perf_counter() - t0
    sat = summarize(res, wall)
    sat_px_s = sat["mpix_per_s"] * 1e6
    mean_px = float(np.mean([r.pixels for r in sat_reqs]))
    # the rate as a fraction of the 8 TB/s HBM roofline, at the algorithmic
    # bytes of the stack formulation of each request (f, theta-or-f, sigma in,
    # the output out, the N + 2 stack planes written and read once)
    bpp = (sum(r.pixels * (16 + 8 * (r.N + 2)) for r in sat_reqs) /
           sum(r.pixels for r in sat_reqs))
    hbm = lambda mpix_s: round(mpix_s * 1e6 * bpp / 8e12, 4)
    sat["hbm_roofline_frac"] = hbm(sat["mpix_per_s"])
    report = {"saturation": sat, "loads": {}, "breakdown": breakdown(sat_reqs, precision),
              "stack_formulation_bytes_per_pixel": round(bpp, 2)}
    for L in loads:
        rate = L * sat_px_s / mean_px
        reqs = make_requests(seed + int(1000 * L), n + warm, rate, scale=scale)
        srv = Server(ex, budget)
        res = srv.run(reqs)
        report["loads"][str(L)] = summarize(res[warm:])
        report["loads"][str(L)]["offered_req_per_s"] = rate
        report["loads"][str(L)]["hbm_roofline_frac"] = hbm(report["loads"][str(L)]["mpix_per_s"])
    return report


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--warm", type=int, default=30)
    ap.add_argument("--loads", type=float, nargs="+", default=[0.3, 0.6, 0.9])
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--scale", type=float, default=1.0)
    a = ap.parse_args()
    print(json.dumps(bench(a.loads, a.requests, a.warm, a.slots, a.budget_gb,
                           precision=a.precision, scale=a.scale)), flush=True)
