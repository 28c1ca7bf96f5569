"""Serving simulations as they arrive (continuous batching).

Requests of different sizes and parameters arrive by a Poisson process.  A
single scheduler loop admits them, first come first served, into a batch
whose device workspace is a fixed budget (admission by HBM footprint: a
request waits while no free region is large enough or no slot is free),
advances everything admitted in chunks of `chunk` steps (one batched launch
per kernel type, replayed from captured graphs), polls for finished
requests, releases their slots and records the latency from arrival to the
moment the final fields are ready on the device.  Requests that arrive while
others run join at the next chunk boundary, so their work overlaps on the
device; each one computes exactly what it would compute alone.  A request
whose footprint exceeds the whole budget is refused (listed in the
summary) rather than waited for.
"""

import collections
import time

import numpy as np

from .workloads import five_smooth_at_least

SIZES = (64, 128, 256, 512)
SIZE_WEIGHTS = (0.4, 0.3, 0.2, 0.1)


def make_requests(n, rate=50.0, seed=181205711, steps=5000, sizes=SIZES, weights=SIZE_WEIGHTS,
                  T_range=(120.0, 400.0), C_choices=(1.0, 10.0, 100.0), precision="fp32_f64math"):
    """Seeded request stream: arrival times (exponential gaps of mean 1/rate
    seconds) and the parameters of each simulation."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for i in range(n):
        ny = int(rng.choice(sizes, p=weights))
        out.append(dict(id=i, arrival=float(t[i]), steps=int(steps),
                        params=dict(nx=five_smooth_at_least(round(1.22 * ny)), ny=ny,
                                    T=float(rng.uniform(*T_range)), C=float(rng.choice(C_choices)), M=10.0,
                                    Fe=4000.0, tau_plus=0.8, Lambda=0.25, Lambda_g=1e-6, noise_amp=1e-3,
                                    seed=seed, instance_id=i, precision=precision)))
    return out


class BatchBackend:
    """The HIP batch (C ABI lbm_ec_batch_*) behind the scheduler."""

    def __init__(self, budget_bytes, max_slots=256, precision="fp32_f64math", device="cuda:0", tuning=None,
                 keep=()):
        from .lbm_ec import Batch

        self.batch = Batch(max_slots, budget_bytes, precision=precision, emit_every=0, hist_rows=1, device=device)
        if tuning is not None:
            self.batch.set_tuning(*tuning)
        self.keep = set(keep)
        self.kept = {}

    def admit(self, req):
        return self.batch.admit(req["steps"], **req["params"])

    def step(self, n):
        self.batch.step(n)

    def poll(self):
        return self.batch.poll()

    def finish(self, slot, req):
        """Releases a finished slot; returns the health of its final state
        (no non-finite moments, rho > 0) from the slot's last history row."""
        if req["id"] in self.keep:
            self.kept[req["id"]] = {k: v.cpu().numpy() for k, v in self.batch.fields(slot).items()}
        healthy = bool(self.batch.history(slot)[-1, 5] == 0)
        self.batch.release(slot)
        return {"healthy": healthy}

    def close(self):
        self.batch.close()


def serve(requests, backend, chunk=100, warmup=0, clock=time.perf_counter, sleep=time.sleep, max_wall=None):
    """Runs the stream to completion.  Returns per-request records and the
    summary (p50 / p99 latency over requests after `warmup`, runs/s)."""
    pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
    waiting = collections.deque()
    running = {}
    records = []
    refused = []
    queued_max = 0
    t0 = clock()
    while pending or waiting or running:
        now = clock() - t0
        if max_wall is not None and now > max_wall:
            raise TimeoutError("serving did not finish within max_wall")
        while pending and pending[0]["arrival"] <= now:
            waiting.append(pending.popleft())
        while waiting:
            req = waiting[0]
            slot = backend.admit(req)
            if slot is None:
                if running:
                    break  # no slot or no room: wait for a release
                # nothing runs, so the whole budget is free: this request
                # can never be admitted
                waiting.popleft()
                refused.append(req["id"])
                continue
            waiting.popleft()
            req["admitted"] = clock() - t0
            running[slot] = req
        queued_max = max(queued_max, len(waiting))
        if running:
            backend.step(chunk)
            done = backend.poll()
            t_done = clock() - t0
            for slot in done:
                req = running.pop(slot)
                extra = backend.finish(slot, req) or {}
                records.append(dict(id=req["id"], arrival=req["arrival"], admitted=req["admitted"], done=t_done,
                                    latency=t_done - req["arrival"], nodes=req["params"]["nx"] * req["params"]["ny"],
                                    steps=req["steps"], **extra))
        elif pending:
            sleep(max(0.0, pending[0]["arrival"] - (clock() - t0)))
    wall = clock() - t0
    lat = np.array([r["latency"] for r in records if r["id"] >= warmup])
    node_steps = sum(r["nodes"] * r["steps"] for r in records)
    summary = dict(requests=len(records), wall_s=wall, runs_per_s=len(records) / wall,
                   p50_s=float(np.percentile(lat, 50)) if len(lat) else None,
                   p99_s=float(np.percentile(lat, 99)) if len(lat) else None,
                   mean_s=float(lat.mean()) if len(lat) else None,
                   mlups=node_steps / wall / 1e6, max_queue=queued_max, refused=refused,
                   unhealthy=sum(1 for r in records if r.get("healthy") is False))
    return records, summary
