"""Continuous (iteration-level) batching on the GPU: each request's output
bits are the same alone and in the mix.

Small-ring analogs of the two serving nets (the MNIST-shaped net: FFConv +
x^2, CP->DP combine, FC; the CIFAR-shaped net: two FFConv stages over two
DensePack input ciphertexts) run through their engines with requests
admitted at different ticks, so chains of different requests, layers and
step indices share launches and the two classes' ticks interleave on one
stream.  Every output must equal the output of the same request run alone
through the one-call net (EncryptedNet.forward), bit for bit, and decrypt to
the FP64 forward pass.  The same mix also runs through the serving loop
(ContinuousServer with device events).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402


def _setup(name):
    from paper_2102_03494_amd import nets
    from paper_2102_03494_amd.client import Client
    from paper_2102_03494_amd.he import HEContext
    if name == "mnist":
        spec = nets.mnist_spec(n=1024, q_bits=(30,) * 5, p_bits=40, image=8, d=3, stride=2, pad=1, r=2, o_c=3,
                               fc_out=4)
    else:
        spec = nets.cifar_spec(n=1024, q_bits=(30,) * 6, p_bits=40, image=8, c_in=3, r1=2, o1=16, r2=2, o2=16)
    ctx = HEContext(spec.n, spec.q_bits, spec.p_bits)
    weights = nets.net_weights(spec)
    net = nets.EncryptedNet(ctx, spec, weights)
    cl = Client(ctx, spec.workload)
    cl.gen_rotation_keys(net.rotation_steps())
    cl.gen_relin_key()
    ctx.reserve(net.workspace_need(4) + (64 << 20))
    return spec, weights, net, cl


def _requests(spec, net, cl, cls, rids):
    from paper_2102_03494_amd.serve import Request
    g = spec.stages[0].geom
    reqs = []
    for rid in rids:
        x = synth.image("serving", (g.h, g.w, g.c_in), index=rid)
        cts = [cl.encrypt(v, spec.level, spec.scale, index=10_000 + rid).data[0] for v in net.input_layout(x)]
        reqs.append(Request(rid, cls, 0.0, payload=torch.stack(cts)))
    return reqs


def _engines(mnist, cifar):
    from paper_2102_03494_amd.engine import NetEngine
    em = NetEngine(mnist[2], 8 << 30, max_inflight=8, max_admit=2)
    # the CIFAR-shaped engine advances at most 64 chains per tick in blocks of 48
    ec = NetEngine(cifar[2], 8 << 30, max_inflight=8, max_admit=1, max_chains=64, chain_block=48)
    for e in (em, ec):
        e.ctx.reserve(e.workspace_need())
    return em, ec


def _check_alone(setup, eng, reqs):
    from paper_2102_03494_amd.he import Ct
    spec, weights, net, cl = setup
    from paper_2102_03494_amd import nets
    for r in reqs:
        alone = net.forward(r.payload[None])
        torch.cuda.synchronize()
        out, i = eng.outputs[r.rid]
        assert torch.equal(out[i], alone.data[0]), (r.cls, r.rid)
        g = spec.stages[0].geom
        x = synth.image("serving", (g.h, g.w, g.c_in), index=r.rid)
        ref = nets.reference_forward(spec, weights, x)
        if spec.fc is None:
            ref = ref.reshape(-1, ref.shape[-1])
        got = net.decode(cl, Ct(out, eng.out_scale), i)
        assert np.abs(got - ref.reshape(got.shape)).max() < 1e-3, (r.cls, r.rid)


def test_engine_mix_bits_equal_alone():
    mnist, cifar = _setup("mnist"), _setup("cifar")
    em, ec = _engines(mnist, cifar)
    rm = _requests(mnist[0], mnist[2], mnist[3], "mnist", [1, 2, 3, 4, 5])
    rc = _requests(cifar[0], cifar[2], cifar[3], "cifar", [11, 12])
    # staggered arrivals: requests join while others are mid-layer
    plan = {0: ([rm[0]], [rc[0]]), 3: ([rm[1], rm[2]], []), 7: ([], [rc[1]]), 11: ([rm[3]], []), 20: ([rm[4]], [])}
    done = []
    tick = 0
    mixed = False
    while tick < 2000:
        add_m, add_c = plan.get(tick, ([], []))
        for r in add_m:
            em.submit(r)
        for r in add_c:
            ec.submit(r)
        got_m = em.tick()
        got_c = ec.tick()
        done += (got_m or []) + (got_c or [])
        if em.inflight >= 2 or ec.inflight >= 2:
            mixed = True
        tick += 1
        if tick > max(plan) and not em.has_work() and not ec.has_work():
            break
    torch.cuda.synchronize()
    assert mixed and len(done) == 7
    assert em.stats.admitted == 5 and ec.stats.admitted == 2
    _check_alone(mnist, em, rm)
    _check_alone(cifar, ec, rc)


def test_continuous_server_mix_bits_equal_alone():
    from paper_2102_03494_amd.serve import ContinuousServer
    mnist, cifar = _setup("mnist"), _setup("cifar")
    em, ec = _engines(mnist, cifar)
    rm = _requests(mnist[0], mnist[2], mnist[3], "mnist", [21, 22, 23, 24])
    rc = _requests(cifar[0], cifar[2], cifar[3], "cifar", [31, 32])
    for k, r in enumerate(rm):
        r.t_arrival = 0.002 * k
    for k, r in enumerate(rc):
        r.t_arrival = 0.001 + 0.003 * k
    stream = torch.cuda.Stream()

    def mark(cls):
        ev = torch.cuda.Event()
        ev.record(stream)
        return ev

    server = ContinuousServer({"mnist": em, "cifar": ec}, mark, lambda ev: ev.query(), order=["mnist", "cifar"])
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        rep = server.run(rm + rc, window_s=1.0, cap_s=60.0)
    torch.cuda.synchronize()
    assert rep["classes"]["mnist"]["completed"] == 4 and rep["classes"]["cifar"]["completed"] == 2
    assert rep["backlog_at_end"] == 0
    _check_alone(mnist, em, rm)
    _check_alone(cifar, ec, rc)
