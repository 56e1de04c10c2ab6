"""Iteration-level (continuous) batching of the encrypted nets.

The serving nets spend nearly all their time in the rotate-and-add chains of
their DensePack layers (Table I: R rotations per dot product; the DensePack
outputs of a layer are independent chains).  Instead of running whole
batches of requests through a net one after another, an engine keeps every
in-flight request's chains together and advances them in shared launches:

* a request's net is a plan of DensePack layers (each FFConv stage's W1,
  and the MNIST-shaped net's FC layer); a layer runs as
  HMA (he_densepack_hma) -> R rotate-and-add steps -> finish (for FFConv the
  rescale, gather, 1x1 ConvPack, rescale and x^2 of ffconv_tail_batch, then
  the CP->DP combine when another layer follows; for the FC layer a
  rescale), and the finish starts the next layer's HMA;
* each tick of the engine (1) finishes the layers whose chains are done,
  (2) admits waiting requests whose accumulators fit the HBM budget (their
  first layer's HMA), (3) runs ONE rotate-and-add step for chains of every
  in-flight request, whatever its layer and step index, in one ragged launch
  chain (he_rotsum_groups: each group its own Galois element and key);
* a per-tick chain budget bounds how long a tick occupies the GPU, so a
  server can interleave the ticks of engines on different rings (the
  MNIST-shaped and CIFAR-shaped classes) on one stream without one class's
  large layers holding the other's short steps for a whole layer.

Every ciphertext's arithmetic is the same as in the one-call layers
(ffconv_layer_batch, he_conv_densepack_batch), so each request's output bits
are the same alone, in a batch, or in the mix.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from .he import Ct


@dataclass
class _Chains:
    acc: torch.Tensor  # [count][2][level][N], a slice of its run's accumulators
    step: int = 0


@dataclass
class _LayerRun:
    reqs: list
    layer: int
    acc: torch.Tensor
    chains: list
    seq: int
    bytes: int


@dataclass
class EngineStats:
    admitted: int = 0
    ticks: int = 0
    steps: int = 0
    chain_steps: int = 0
    peak_inflight: int = 0
    peak_bytes: int = 0
    deferrals: int = 0


class NetEngine:
    """Continuous batching of one FFConv net (EncryptedNet, not the plain
    variant) on its context.

    max_chains: chains advanced per tick (None: all); chain_block: chains per
    group (a layer's accumulators are split into blocks that advance
    independently, so a tick can take part of a large layer); budget_bytes:
    HBM for in-flight accumulators; max_inflight: request slots; max_admit:
    requests admitted per tick (they share one HMA launch)."""

    def __init__(self, net, budget_bytes: int, max_inflight: int = 64, max_admit: int = 32,
                 max_chains: int | None = None, chain_block: int | None = None, keep_outputs: int | None = None):
        if net.plain:
            raise ValueError("the engine runs FFConv nets")
        self.net, self.ctx = net, net.ctx
        self.budget, self.max_inflight, self.max_admit = budget_bytes, max_inflight, max_admit
        self.max_chains, self.chain_block = max_chains, chain_block
        self.r_steps = net.r_steps
        self.waiting = []
        self.runs = []
        self.inflight = 0
        self.bytes = 0
        self.seq = 0
        self.stats = EngineStats()
        self.outputs = {}  # rid -> (tensor, index), for the first keep_outputs requests (None: all)
        self.keep_outputs = keep_outputs
        self._layers = self._plan()

    # ---- plan ------------------------------------------------------------------
    def _plan(self):
        """Per DensePack layer: (desc, filters, level, outputs per request, kind)."""
        n = self.ctx.n
        layers = []
        for k, rec in enumerate(self.net.stages):
            g = rec["spec"].geom
            layers.append(dict(kind="ffconv", k=k, desc=rec["desc"], filt=rec["filt"], level=rec["level"],
                               outs=g.spatial * rec["spec"].r))
        if self.net.fc is not None:
            fc = self.net.fc
            layers.append(dict(kind="fc", desc=fc["desc"], filt=fc["filt"], level=fc["level"],
                               outs=fc["desc"].o_c))
        for ly in layers:
            ly["bytes"] = ly["outs"] * 2 * ly["level"] * n * 8
        return layers

    @property
    def out_scale(self) -> float:
        net = self.net
        return net.fc["out_scale"] if net.fc is not None else net.stages[-1]["out_scale"]

    def request_bytes(self) -> int:
        """HBM one request holds while in flight: its largest layer's
        accumulators, plus that layer's output."""
        return max(ly["bytes"] for ly in self._layers) * 2

    def workspace_need(self) -> int:
        """Context workspace for a tick: the key switch of up to max_chains
        chains and the finish of max_admit requests."""
        ctx = self.ctx
        level0 = self._layers[0]["level"]
        chains = self.max_chains or self.max_admit * self._layers[0]["outs"]
        need = ctx.workspace_need(min(chains, 16000), level0)
        return max(need, self.net.workspace_need(self.max_admit))

    # ---- queue -----------------------------------------------------------------
    def submit(self, req):
        self.waiting.append(req)

    def has_work(self) -> bool:
        return bool(self.waiting) or bool(self.runs)

    def backlog(self) -> int:
        return len(self.waiting) + self.inflight

    # ---- one iteration ------------------------------------------------------------
    def _start(self, reqs, layer: int, xs: torch.Tensor):
        ly = self._layers[layer]
        xs = xs.contiguous()
        if xs.dim() == 4:  # [B][2][level][N] -> [B][1][2][level][N]
            xs = xs.unsqueeze(1)
        acc = self.ctx.densepack_hma(xs, ly["desc"], ly["filt"])
        block = self.chain_block or acc.shape[0]
        chains = [_Chains(acc[i:i + block]) for i in range(0, acc.shape[0], block)]
        run = _LayerRun(reqs, layer, acc, chains, self.seq, len(reqs) * ly["bytes"])
        self.seq += 1
        self.runs.append(run)
        self.bytes += run.bytes

    def _finish(self, run):
        """Finish a layer; returns the requests whose net is done."""
        ctx, net = self.ctx, self.net
        ly = self._layers[run.layer]
        b = len(run.reqs)
        self.runs.remove(run)
        self.bytes -= run.bytes
        if ly["kind"] == "ffconv":
            rec = net.stages[ly["k"]]
            st = rec["spec"]
            z = ctx.ffconv_tail_batch(run.acc, b, rec["desc"], rec["mask"], net._w2_tabs(ly["k"], b), st.o_c,
                                      st.square)
            if "per_dense" in rec:
                nxt = ctx.combine_cp_dp_batch(Ct(z, rec["out_scale"]), st.geom.spatial, rec["per_dense"]).data
            else:
                nxt = z
        else:
            y = ctx.rescale(Ct(run.acc, 1.0)).data
            nxt = y.view(b, ly["outs"], 2, ly["level"] - 1, ctx.n)
        if run.layer + 1 < len(self._layers):
            self._start(run.reqs, run.layer + 1, nxt)
            return []
        for i, r in enumerate(run.reqs):
            if self.keep_outputs is None or len(self.outputs) < self.keep_outputs:
                self.outputs[r.rid] = (nxt, i)
        self.inflight -= b
        return list(run.reqs)

    def tick(self) -> list | None:
        """Enqueue one iteration on the current stream.  Returns the requests
        whose outputs this iteration completes (possibly empty), or None when
        nothing was enqueued."""
        issued = False
        done = []
        for run in [r for r in self.runs if all(c.step >= self.r_steps for c in r.chains)]:
            done += self._finish(run)
            issued = True
        # admission by slots and HBM budget, oldest first
        per = self.request_bytes()
        admit = []
        while (self.waiting and len(admit) < self.max_admit and self.inflight + len(admit) < self.max_inflight
               and self.bytes + per * (len(admit) + 1) <= self.budget):
            admit.append(self.waiting.pop(0))
        if self.waiting:
            self.stats.deferrals += len(self.waiting)
        if admit:
            xs = torch.stack([r.payload for r in admit])
            self.inflight += len(admit)
            self.stats.admitted += len(admit)
            self._start(admit, 0, xs)
            issued = True
        # one rotate-and-add step for chains of every in-flight layer, oldest first
        left = self.max_chains if self.max_chains is not None else math.inf
        groups = []
        for run in sorted(self.runs, key=lambda r: r.seq):
            for ch in run.chains:
                cnt = ch.acc.shape[0]
                if ch.step < self.r_steps and (cnt <= left or not groups):
                    groups.append(ch)
                    left -= cnt
        if groups:
            self.ctx.rotsum_groups([(ch.acc, ch.step) for ch in groups])
            for ch in groups:
                ch.step += 1
            self.stats.steps += 1
            self.stats.chain_steps += sum(ch.acc.shape[0] for ch in groups)
            issued = True
        if not issued:
            return None
        self.stats.ticks += 1
        self.stats.peak_inflight = max(self.stats.peak_inflight, self.inflight)
        self.stats.peak_bytes = max(self.stats.peak_bytes, self.bytes)
        return done

    def drain(self) -> list:
        """Run ticks until every submitted request is done (for tests and
        calibration); returns the requests in completion order."""
        out = []
        while self.has_work():
            got = self.tick()
            if got is None:
                break
            out += got
        return out
