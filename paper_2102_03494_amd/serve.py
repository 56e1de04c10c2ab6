"""Encrypted-inference serving loop (the paper's MLaaS setting, Sec. 1).

Clients encrypt their images and send them; the server evaluates the net on
the ciphertexts with its plaintext weights and returns encrypted
predictions.  This module runs that server over a seeded arrival stream:

* arrivals: a Poisson process (exponential inter-arrival times) with a
  Bernoulli class flag per request (MNIST-shaped or CIFAR-shaped net);
* queues: one FIFO per class; a request is admitted into a batch when it has
  arrived and the batch's workspace fits the class's HBM budget;
* execution: each class has its own context (its own workspace) and HIP
  stream with at most one batch in flight; by default one batch runs at a
  time (serial), and with `concurrent` the classes' batches overlap on their
  streams.  Measured on MI355X, overlapping hurts the short class: the
  CIFAR-shaped kernels (tens of thousands of workgroups each) hold the CUs
  and every dependent MNIST-shaped kernel queues behind them, so serial
  shortest-class-first gives the lower latencies; completion is polled with
  stream events either way;
* policy "sjf" starts the class with the cheaper requests first (by a
  measured cost per request), "fifo" the class whose head arrived first; a
  batch takes up to max_batch requests of one class, and all requests of a
  batch run one model, so each layer is one batched library call;
* every request waiting when a batch is formed but not admitted to it counts
  one deferral; the run stops admitting at the end of the arrival window and
  drains until a time cap, and what is left is reported as backlog.

Latency is completion minus arrival, on the host clock, with the GPU work of
each batch synchronised before its requests complete.  Client-side encoding,
encryption and decryption happen outside the clock.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from collections import deque
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    cls: str
    t_arrival: float
    payload: object = None
    t_done: float | None = None
    deferrals: int = 0
    batch_id: int = -1


@dataclass
class ClassStats:
    offered: int = 0
    completed: int = 0
    batches: int = 0
    admitted: int = 0
    deferrals: int = 0
    latencies: list = field(default_factory=list)
    busy_s: float = 0.0


def percentile(xs, q: float) -> float | None:
    """q-th percentile (0..100) by linear interpolation between order statistics."""
    if not xs:
        return None
    s = sorted(xs)
    pos = (len(s) - 1) * q / 100.0
    lo = math.floor(pos)
    hi = min(lo + 1, len(s) - 1)
    return s[lo] + (s[hi] - s[lo]) * (pos - lo)


class Scheduler:
    """Admission, batching and accounting; the executors do the work.

    executors[cls] must provide max_batch (int), fits(b) -> bool (the batch's
    workspace fits the class's HBM budget), cost_per_request (seconds, for
    the sjf policy), start(requests) -> handle (enqueues the batch) and
    done(handle) -> bool.  now() and sleep(dt) are the clock, injectable for
    tests; poll_s is the sleep between completion polls.
    """

    def __init__(self, executors: dict, policy: str = "sjf", now=time.perf_counter, sleep=time.sleep,
                 poll_s: float = 2e-4, concurrent: bool = False):
        if policy not in ("sjf", "fifo"):
            raise ValueError(policy)
        self.ex, self.policy, self.now, self.sleep, self.poll = executors, policy, now, sleep, poll_s
        self.concurrent = concurrent

    def _batch_size(self, cls: str, waiting: int) -> int:
        ex = self.ex[cls]
        b = min(waiting, ex.max_batch)
        while b > 0 and not ex.fits(b):
            b -= 1
        return b

    def run(self, requests: list, window_s: float, cap_s: float, progress_s: float = 0.0) -> dict:
        """Serve `requests` (arrival times relative to the start); with
        progress_s > 0, print completed counts and backlog to stderr every
        progress_s seconds."""
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        queues = {c: deque() for c in self.ex}
        stats = {c: ClassStats() for c in self.ex}
        for r in reqs:
            stats[r.cls].offered += 1
        inflight = {}  # cls -> (handle, batch, t_start)
        nxt = 0
        peak_backlog = 0
        rejected = 0
        batch_id = 0
        t0 = self.now()
        next_report = progress_s
        while True:
            t = self.now() - t0
            if progress_s > 0 and t >= next_report:
                next_report += progress_s
                done = {c: st.completed for c, st in stats.items()}
                print(f"# t={t:.0f}s completed {done} backlog {sum(len(q) for q in queues.values())}",
                      file=sys.stderr, flush=True)
            while nxt < len(reqs) and reqs[nxt].t_arrival <= min(t, window_s):
                queues[reqs[nxt].cls].append(reqs[nxt])
                nxt += 1
            for cls, (h, batch, ts) in list(inflight.items()):
                if self.ex[cls].done(h):
                    t_end = self.now() - t0
                    st = stats[cls]
                    st.busy_s += t_end - ts
                    for r in batch:
                        r.t_done = t_end
                        st.completed += 1
                        st.latencies.append(t_end - r.t_arrival)
                    del inflight[cls]
            peak_backlog = max(peak_backlog, sum(len(q) for q in queues.values()))
            if t >= cap_s:
                break
            idle = [c for c, q in queues.items() if q and c not in inflight]
            if self.policy == "sjf":
                idle.sort(key=lambda c: (self.ex[c].cost_per_request, queues[c][0].t_arrival))
            else:
                idle.sort(key=lambda c: queues[c][0].t_arrival)
            if not self.concurrent and inflight:
                idle = []
            for cls in idle:
                if not self.concurrent and inflight:
                    break
                q = queues[cls]
                b = self._batch_size(cls, len(q))
                while b == 0 and q:  # not even one request fits the budget: it can never run
                    q.popleft()
                    rejected += 1
                    b = self._batch_size(cls, len(q))
                if b == 0:
                    continue
                batch = [q.popleft() for _ in range(b)]
                for c2, q2 in queues.items():
                    for r in q2:
                        r.deferrals += 1
                        stats[c2].deferrals += 1
                for r in batch:
                    r.batch_id = batch_id
                batch_id += 1
                stats[cls].batches += 1
                stats[cls].admitted += b
                inflight[cls] = (self.ex[cls].start(batch), batch, self.now() - t0)
            if not inflight and not any(queues.values()):
                if nxt >= len(reqs) or reqs[nxt].t_arrival > window_s:
                    break
                self.sleep(max(0.0, min(reqs[nxt].t_arrival, cap_s) - t))
            else:
                self.sleep(self.poll)
        makespan = self.now() - t0
        out = {"policy": self.policy, "window_s": window_s, "cap_s": cap_s, "makespan_s": makespan,
               "peak_backlog": peak_backlog, "rejected": rejected,
               "backlog_at_end": sum(len(q) for q in queues.values()) + sum(len(v[1]) for v in inflight.values())
               + sum(1 for r in reqs[nxt:] if r.t_arrival <= window_s),
               "classes": {}}
        for c, st in stats.items():
            out["classes"][c] = {
                "offered": st.offered, "completed": st.completed, "batches": st.batches,
                "admitted": st.admitted, "deferrals": st.deferrals,
                "p50_latency_s": percentile(st.latencies, 50), "p99_latency_s": percentile(st.latencies, 99),
                "completed_per_s": st.completed / makespan if makespan > 0 else None,
                "gpu_busy_s": st.busy_s,
            }
        total = sum(st.completed for st in stats.values())
        out["completed"] = total
        out["completed_per_s"] = total / makespan if makespan > 0 else None
        out["p50_latency_s"] = percentile([x for st in stats.values() for x in st.latencies], 50)
        out["p99_latency_s"] = percentile([x for st in stats.values() for x in st.latencies], 99)
        return out


class ContinuousServer:
    """Continuous batching across classes: each class is an engine
    (engine.NetEngine) that advances every in-flight request by one step per
    tick, and arrivals join their engine's next tick (as slots and HBM free
    up) instead of waiting for a batch to drain.  The server interleaves the
    engines' ticks in `order` (round robin; repeat a class to weight it) on
    one stream, keeping at most `ahead` ticks enqueued beyond the GPU, and
    completes a request when the tick that produced its output has finished
    on the device.

    engines[cls] provides submit(req), has_work(), backlog(), tick() -> list
    of requests its enqueued work completes, or None when it enqueued
    nothing; mark(cls) returns a token recorded after the work just enqueued
    and done(token) tells whether it has run.  now() and sleep(dt) are the
    clock (injectable for tests)."""

    def __init__(self, engines: dict, mark, done, now=time.perf_counter, sleep=time.sleep, poll_s: float = 2e-4,
                 ahead: int = 2, order=None):
        self.ex, self.mark, self.done, self.now, self.sleep, self.poll = engines, mark, done, now, sleep, poll_s
        self.ahead = ahead
        self.order = list(order) if order else list(engines)

    def run(self, requests: list, window_s: float, cap_s: float, progress_s: float = 0.0) -> dict:
        reqs = sorted(requests, key=lambda r: r.t_arrival)
        stats = {c: ClassStats() for c in self.ex}
        for r in reqs:
            stats[r.cls].offered += 1
        pending = deque()  # (token, cls, requests completed by that tick)
        nxt = 0
        rr = 0
        peak_backlog = 0
        t0 = self.now()
        next_report = progress_s
        while True:
            t = self.now() - t0
            if progress_s > 0 and t >= next_report:
                next_report += progress_s
                done = {c: st.completed for c, st in stats.items()}
                print(f"# t={t:.0f}s completed {done} backlog {sum(e.backlog() for e in self.ex.values())}",
                      file=sys.stderr, flush=True)
            while nxt < len(reqs) and reqs[nxt].t_arrival <= min(t, window_s):
                self.ex[reqs[nxt].cls].submit(reqs[nxt])
                stats[reqs[nxt].cls].admitted += 1
                nxt += 1
            while pending and self.done(pending[0][0]):
                _, cls, fin = pending.popleft()
                t_end = self.now() - t0
                st = stats[cls]
                for r in fin:
                    r.t_done = t_end
                    st.completed += 1
                    st.latencies.append(t_end - r.t_arrival)
            peak_backlog = max(peak_backlog, sum(e.backlog() for e in self.ex.values()))
            if t >= cap_s:
                break
            if len(pending) < self.ahead:
                issued = False
                for k in range(len(self.order)):
                    cls = self.order[(rr + k) % len(self.order)]
                    eng = self.ex[cls]
                    if not eng.has_work():
                        continue
                    fin = eng.tick()
                    if fin is None:
                        continue
                    pending.append((self.mark(cls), cls, fin))
                    stats[cls].batches += 1
                    rr = (rr + k + 1) % len(self.order)
                    issued = True
                    break
                if issued:
                    continue
            if not pending and not any(e.has_work() for e in self.ex.values()):
                if nxt >= len(reqs) or reqs[nxt].t_arrival > window_s:
                    break
                self.sleep(max(0.0, min(reqs[nxt].t_arrival, cap_s) - t))
            else:
                self.sleep(self.poll)
        makespan = self.now() - t0
        out = {"mode": "continuous", "window_s": window_s, "cap_s": cap_s, "makespan_s": makespan,
               "peak_backlog": peak_backlog,
               "backlog_at_end": sum(e.backlog() for e in self.ex.values())
               + sum(1 for r in reqs[nxt:] if r.t_arrival <= window_s),
               "classes": {}}
        for c, st in stats.items():
            out["classes"][c] = {
                "offered": st.offered, "completed": st.completed, "ticks": st.batches, "arrived": st.admitted,
                "p50_latency_s": percentile(st.latencies, 50), "p99_latency_s": percentile(st.latencies, 99),
                "completed_per_s": st.completed / makespan if makespan > 0 else None,
                "backlog_at_end": self.ex[c].backlog(),
            }
        total = sum(st.completed for st in stats.values())
        out["completed"] = total
        out["completed_per_s"] = total / makespan if makespan > 0 else None
        out["p50_latency_s"] = percentile([x for st in stats.values() for x in st.latencies], 50)
        out["p99_latency_s"] = percentile([x for st in stats.values() for x in st.latencies], 99)
        return out


class NetExecutor:
    """Runs batches of one class on its own context and net."""

    def __init__(self, net, budget_bytes: int, max_batch: int, keep: int = 3):
        import torch
        self.net, self.budget, self.max_batch, self.keep = net, budget_bytes, max_batch, keep
        self.torch = torch
        self._need = {}
        self.cost_per_request = 1.0
        self.kept = {}
        self.stream = torch.cuda.Stream()  # default priority
        b = max_batch
        while b > 0 and not self.fits(b):
            b -= 1
        self.max_batch = b
        if b > 0:
            net.ctx.reserve(self.need(b))

    def need(self, b: int) -> int:
        """Workspace bytes of a batch of b (reserved once, for max_batch)."""
        if b not in self._need:
            self._need[b] = self.net.workspace_need(b)
        return self._need[b]

    def fits(self, b: int) -> bool:
        return self.need(b) + self.net.activation_bytes(b) <= self.budget

    def start(self, batch):
        """Enqueues the batch on this class's stream; returns (event, output)."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            xs = torch.stack([r.payload for r in batch]).contiguous()
            out = self.net.forward(xs)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        for i, r in enumerate(batch):
            if len(self.kept) < self.keep:
                self.kept[r.rid] = (out, i)
        return ev, out, xs

    def done(self, handle) -> bool:
        return handle[0].query()

    def calibrate(self, sample_payload, reps: int = 1):
        """Measured seconds per request of one full batch (the sjf cost)."""
        torch = self.torch
        b = max(1, self.max_batch)
        torch.cuda.synchronize()
        with torch.cuda.stream(self.stream):
            xs = torch.stack([sample_payload] * b).contiguous()
            self.net.forward(xs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(self.stream):
            for _ in range(reps):
                self.net.forward(xs)
        torch.cuda.synchronize()
        self.cost_per_request = (time.perf_counter() - t0) / reps / b
        return self.cost_per_request


def build_class(name: str, variant: str, budget_gb: float, max_batch: int, small: bool = False):
    """Context, keys, net and client of one class."""
    from . import nets
    from .client import Client
    from .he import HEContext
    spec = nets.mnist_spec() if name == "mnist" else nets.cifar_spec()
    ctx = HEContext(spec.n, spec.q_bits, spec.p_bits)
    weights = nets.net_weights(spec)
    if variant == "tap":
        net = nets.TapNet(ctx, spec, weights)
    else:
        net = nets.EncryptedNet(ctx, spec, weights, plain=(variant == "plain"))
    client = Client(ctx, spec.workload)
    client.gen_rotation_keys(net.rotation_steps())
    if net.needs_relin():
        client.gen_relin_key()
    ex = NetExecutor(net, int(budget_gb * (1 << 30)), max_batch)
    return spec, weights, net, client, ex


def build_engine(name: str, budget_gb: float, small: bool = False):
    """Context, keys, net, client and continuous-batching engine of one class
    (FFConv net).  The MNIST-shaped class advances all its chains every tick
    and admits up to 32 requests per tick; the CIFAR-shaped class advances at
    most 2048 chains per tick (about one N = 16384 key-switch launch of
    2048 ciphertexts), so its ticks stay short beside the other class's, and
    keeps two requests in flight (one request's layer already fills a tick,
    so more in flight would only stretch every one's latency)."""
    from . import nets
    from .client import Client
    from .engine import NetEngine
    from .he import HEContext
    spec = nets.mnist_spec() if name == "mnist" else nets.cifar_spec()
    ctx = HEContext(spec.n, spec.q_bits, spec.p_bits)
    weights = nets.net_weights(spec)
    net = nets.EncryptedNet(ctx, spec, weights, plain=False)
    client = Client(ctx, spec.workload)
    client.gen_rotation_keys(net.rotation_steps())
    if net.needs_relin():
        client.gen_relin_key()
    budget = int(budget_gb * (1 << 30))
    if name == "mnist":
        eng = NetEngine(net, budget, max_inflight=256, max_admit=32, keep_outputs=8)
    else:
        eng = NetEngine(net, budget, max_inflight=2, max_admit=1, max_chains=2048, chain_block=2048, keep_outputs=8)
    ctx.reserve(eng.workspace_need())
    return spec, weights, net, client, eng


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--window", type=float, default=10.0, help="arrival window (s)")
    ap.add_argument("--rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--p-mnist", type=float, default=0.7, help="probability that a request is MNIST-shaped")
    ap.add_argument("--cap", type=float, default=120.0, help="stop draining after this many seconds")
    ap.add_argument("--variant", choices=("ffconv", "plain", "tap"), default="ffconv",
                    help="ffconv: FFConv nets (DensePack W1); plain: composed-weight DensePack convs; tap: FFConv "
                         "nets with tap-style W1 (hoisted tap rotations), served in whole-request batches")
    ap.add_argument("--policy", choices=("sjf", "fifo"), default="sjf")
    ap.add_argument("--budget-gb", type=float, default=120.0, help="HBM workspace budget per class")
    ap.add_argument("--max-batch-mnist", type=int, default=32)
    ap.add_argument("--max-batch-cifar", type=int, default=2)
    ap.add_argument("--classes", default="mnist,cifar")
    ap.add_argument("--concurrent", action="store_true", help="overlap the classes' batches on their streams")
    ap.add_argument("--mode", choices=("continuous", "queue"), default="continuous",
                    help="continuous: iteration-level batching (the ffconv variant; the others always run as "
                         "queue); queue: batches of whole requests")
    ap.add_argument("--out", default=None)
    return ap.parse_args(argv)


def run_continuous(args) -> dict:
    """Serving with iteration-level batching (ContinuousServer over one
    NetEngine per class, all on one stream)."""
    import numpy as np
    import torch

    import synth
    from .he import Ct
    torch.cuda.set_device(0)
    classes = [c for c in args.classes.split(",") if c]
    times, first = synth.poisson_arrivals("serving", args.rate, args.window, args.p_mnist)
    reqs = []
    for i, (t, is_mnist) in enumerate(zip(times, first)):
        c = "mnist" if is_mnist else "cifar"
        if c in classes:
            reqs.append(Request(i, c, float(t)))
    built = {c: build_engine(c, args.budget_gb) for c in classes}
    for c in classes:
        print(f"# {c}: context, keys, net and engine ready", file=sys.stderr, flush=True)
    for r in reqs:
        spec, _, net, client, _ = built[r.cls]
        g = spec.stages[0].geom
        x = synth.image("serving", (g.h, g.w, g.c_in), index=r.rid)
        cts = [client.encrypt(v, spec.level, spec.scale, index=10_000 + r.rid).data[0] for v in net.input_layout(x)]
        r.payload = torch.stack(cts)
    stream = torch.cuda.Stream()  # default priority
    torch.cuda.synchronize()

    def mark(cls):
        ev = torch.cuda.Event()
        ev.record(stream)
        return ev

    # the short MNIST-shaped requests get two ticks for every CIFAR-shaped one
    server = ContinuousServer({c: built[c][4] for c in classes}, mark, lambda ev: ev.query(),
                              order=[c for c in ("mnist", "mnist", "cifar") if c in classes])
    print(f"# serving {len(reqs)} requests over {args.window} s (cap {args.cap} s), continuous batching",
          file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        rep = server.run(reqs, args.window, args.cap, progress_s=10.0)
    torch.cuda.synchronize()
    errs = {}
    for c in classes:
        spec, weights, net, client, eng = built[c]
        worst = None
        for rid, (out, i) in list(eng.outputs.items())[:3]:
            g = spec.stages[0].geom
            x = synth.image("serving", (g.h, g.w, g.c_in), index=rid)
            ref = nets_reference(spec, weights, x)
            got = net.decode(client, Ct(out, eng.out_scale), i)
            e = float(np.abs(got - ref.reshape(got.shape)).max())
            worst = e if worst is None else max(worst, e)
        errs[c] = worst
        st = eng.stats
        rep["classes"][c].update(ticks_engine=st.ticks, rotate_steps=st.steps, chain_steps=st.chain_steps,
                                 peak_inflight=st.peak_inflight, peak_accumulator_gb=st.peak_bytes / 2**30,
                                 deferred_request_ticks=st.deferrals)
    rep["decrypted_max_abs_err"] = errs
    rep["variant"] = "ffconv"
    rep["rate_per_s"] = args.rate
    rep["p_mnist"] = args.p_mnist
    del built, reqs, server
    torch.cuda.empty_cache()
    return rep


def run(args) -> dict:
    """One serving run (arguments as parse_args gives them); returns the report."""
    if getattr(args, "mode", "queue") == "continuous" and args.variant == "ffconv":
        return run_continuous(args)
    import numpy as np
    import torch

    import synth
    torch.cuda.set_device(0)
    classes = [c for c in args.classes.split(",") if c]
    times, first = synth.poisson_arrivals("serving", args.rate, args.window, args.p_mnist)
    reqs = []
    for i, (t, is_mnist) in enumerate(zip(times, first)):
        c = "mnist" if is_mnist else "cifar"
        if c in classes:
            reqs.append(Request(i, c, float(t)))
    built = {}
    for c in classes:
        mb = args.max_batch_mnist if c == "mnist" else args.max_batch_cifar
        built[c] = build_class(c, args.variant, args.budget_gb, mb)
        print(f"# {c}: context, keys and net ready; max batch {built[c][4].max_batch}", file=sys.stderr, flush=True)
    # client side, before the clock: encrypt every request's image
    for r in reqs:
        spec, _, net, client, _ = built[r.cls]
        g = spec.stages[0].geom
        x = synth.image("serving", (g.h, g.w, g.c_in), index=r.rid)
        cts = [client.encrypt(v, spec.level, spec.scale, index=10_000 + r.rid).data[0] for v in net.input_layout(x)]
        r.payload = torch.stack(cts)
    for c in classes:
        sample = next(r.payload for r in reqs if r.cls == c)
        cost = built[c][4].calibrate(sample)
        print(f"# {c}: {cost * 1e3:.2f} ms per request at batch {built[c][4].max_batch}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()  # the encrypted inputs exist before the clock starts
    sched = Scheduler({c: built[c][4] for c in classes}, args.policy, concurrent=args.concurrent)
    print(f"# serving {len(reqs)} requests over {args.window} s (cap {args.cap} s)", file=sys.stderr, flush=True)
    rep = sched.run(reqs, args.window, args.cap, progress_s=10.0)
    torch.cuda.synchronize()  # batches still in flight at the cap finish before any decryption
    # accuracy of a few completed requests against the FP64 forward pass
    errs = {}
    for c in classes:
        spec, weights, net, client, ex = built[c]
        worst = 0.0
        for rid, (out, i) in list(ex.kept.items())[:3]:
            g = spec.stages[0].geom
            x = synth.image("serving", (g.h, g.w, g.c_in), index=rid)
            ref = nets_reference(spec, weights, x)
            got = net.decode(client, out, i)
            worst = max(worst, float(np.abs(got - ref.reshape(got.shape)).max()))
        errs[c] = worst if ex.kept else None
    rep["decrypted_max_abs_err"] = errs
    rep["mode"] = "queue"
    rep["variant"] = args.variant
    rep["concurrent"] = args.concurrent
    rep["rate_per_s"] = args.rate
    rep["p_mnist"] = args.p_mnist
    rep["max_batch"] = {c: built[c][4].max_batch for c in classes}
    rep["cost_per_request_s"] = {c: built[c][4].cost_per_request for c in classes}
    del built, reqs, sched  # contexts, keys and workspaces go with their nets
    torch.cuda.empty_cache()
    return rep


def main(argv=None):
    args = parse_args(argv)
    rep = run(args)
    line = json.dumps(rep)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    print(line)
    return rep


def nets_reference(spec, weights, x):
    from . import nets
    h = nets.reference_forward(spec, weights, x)
    if spec.fc is None:  # [H][W][C] -> [S][C]
        h = h.reshape(-1, h.shape[-1])
    return h


if __name__ == "__main__":
    main()
