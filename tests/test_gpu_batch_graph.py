"""Batched FFConv layers and HIP-graph replay on the GPU.

* ffconv_layer_batch over three independent layers (each with its own image,
  W1 and W2) returns, layer by layer, the oracle's bits for that layer run
  alone (the Sec. 4 layer, DP-HI2C-CP with x^2), and the same bits as three
  single ffconv_layer calls.
* A graph captured around ffconv_layer_batch replays to the eager result on
  several replays with eager work and synchronisations in between, and
  follows new inputs written into the captured input buffer.
* Calls that copy host tables refuse to be captured (and leave the context
  usable).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from oracle import conv as C  # noqa: E402
from oracle import params as P  # noqa: E402
from oracle import workloads as Wk  # noqa: E402

W = "unit"
H, WD, CIN, D, STRIDE, PAD = 7, 7, 2, 3, 2, 1
R, OC2, KB, LEVEL = 2, 3, 12, 4


def _he():
    from paper_2102_03494_amd import he
    return he


def _setup():
    he = _he()
    from paper_2102_03494_amd.client import Client
    p = P.Params(1024, (30, 30, 30, 30), 40, 2.0**25)
    rots = [1 << j for j in range(9)]
    octx = Wk.make_context(p, W, rotations=rots, relin=True)
    gctx = he.HEContext(p.n, p.q_bits, p.p_bits, workspace_bytes=1 << 28)
    cl = Client(gctx, W)
    cl.gen_rotation_keys(rots)
    cl.gen_relin_key()
    return p, octx, gctx, cl


def _layer(p, octx, idx):
    """Inputs and the oracle's output bits of layer idx."""
    geom = C.ConvGeom(H, WD, CIN, D, STRIDE, PAD)
    x = synth.image(W, (H, WD, CIN), index=40 + idx)
    w1 = synth.weights(W, 200 + 2 * idx, (D, D, CIN, R), 0.3)
    w2 = synth.weights(W, 201 + 2 * idx, (R, OC2), 0.4)
    ct = Wk.encrypt_slots(octx, C.densepack_slots(x, geom, p.slots)[0], LEVEL, p.scale, W, 40 + idx)
    pts = C.densepack_pt_scale(p, LEVEL, p.scale, p.scale)
    bf = C.densepack_base_filters(p, w1, geom, LEVEL, pts)
    y, _ = C.conv_densepack(p, octx, ct, geom, bf, pts)
    target = C.pre_square_target(p, LEVEL - 2, p.scale)
    ms = C.gather_mask_scale(p, y.level, y.scale, target, KB)
    mask = C.encode_onehot(p, y.level, ms)
    z, _ = C.gather_convpack(p, y, geom.spatial, w2, KB, mask, ms)
    want, _ = C.square_rescale(p, octx, z)
    return dict(ct=ct.c, bf=bf, pts=pts, w2=w2, mask=mask, ms=ms, want=want)


def _host(t):
    torch.cuda.synchronize()
    return _he().to_host(t)


def test_ffconv_layer_batch_bit_exact():
    he = _he()
    p, octx, gctx, cl = _setup()
    layers = [_layer(p, octx, i) for i in range(3)]
    desc = he.HEContext.conv_desc(H, WD, CIN, D, STRIDE, PAD, R, 9)
    xs = he.to_device(np.stack([L["ct"] for L in layers]))
    filts = he.to_device(np.stack([L["bf"] for L in layers]))
    tabs = torch.stack([gctx.int_weight_table(L["w2"], KB, LEVEL - 1) for L in layers])
    mask = he.to_device(layers[0]["mask"])  # the mask depends on the scales only
    assert all(np.array_equal(L["mask"], layers[0]["mask"]) for L in layers)
    need = gctx.ffconv_workspace_need(3, LEVEL, desc, OC2, True)
    assert need > 0
    gctx.reserve(need)
    got = gctx.ffconv_layer_batch(xs, p.scale, desc, filts, layers[0]["pts"], mask, layers[0]["ms"], tabs, OC2, KB,
                                  True)
    bits = _host(got.data)
    counts = gctx.last_counts()
    assert counts["rot"] == 3 * R * 16 * 9 and counts["square"] == 3 * OC2
    for i, L in enumerate(layers):
        assert np.array_equal(bits[i], L["want"].c), i
        single = gctx.ffconv_layer(he.Ct(xs[i:i + 1], p.scale), desc, filts[i], L["pts"], mask, L["ms"], L["w2"], KB,
                                   True)
        assert np.array_equal(_host(single.data), bits[i]), i
    assert abs(got.scale - layers[0]["want"].scale) <= 1e-12 * got.scale


def test_graph_replays_match_eager():
    he = _he()
    p, octx, gctx, cl = _setup()
    layers = [_layer(p, octx, i) for i in range(4)]
    desc = he.HEContext.conv_desc(H, WD, CIN, D, STRIDE, PAD, R, 9)
    xs_a = np.stack([L["ct"] for L in layers[:2]])
    xs_b = np.stack([L["ct"] for L in layers[2:]])
    xs = he.to_device(xs_a)
    filts = he.to_device(np.stack([L["bf"] for L in layers[:2]]))
    tabs = torch.stack([gctx.int_weight_table(L["w2"], KB, LEVEL - 1) for L in layers[:2]])
    mask = he.to_device(layers[0]["mask"])
    gctx.reserve(gctx.ffconv_workspace_need(2, LEVEL, desc, OC2, True))
    out = torch.empty((2, OC2, 2, LEVEL - 3, p.n), dtype=torch.int64, device="cuda")

    def run():
        return gctx.ffconv_layer_batch(xs, p.scale, desc, filts, layers[0]["pts"], mask, layers[0]["ms"], tabs,
                                       OC2, KB, True, out=out)

    run()
    eager = _host(out).copy()
    out.zero_()
    graph, _ = gctx.capture(run)
    torch.cuda.synchronize()
    assert not np.array_equal(_host(out), eager)  # capture records, it does not run
    for rep in range(3):
        out.fill_(-1)
        graph.launch()
        assert np.array_equal(_host(out), eager), rep
        # eager work on the same context between replays
        gctx.rotate(he.Ct(xs[0].clone(), p.scale), 1)
        torch.cuda.synchronize()
    # new inputs in the captured buffer: the replay follows them (filters
    # and W2 stay those of layers 0-1, so compare against an eager run)
    xs.copy_(he.to_device(xs_b))
    graph.launch()
    replay_b = _host(out).copy()
    run()
    assert np.array_equal(_host(out), replay_b)
    assert not np.array_equal(replay_b, eager)
    graph.close()


def test_host_table_calls_refuse_capture():
    he = _he()
    p, octx, gctx, cl = _setup()
    w = np.ones((2, 3))
    buf = torch.empty(24, dtype=torch.int64, device="cuda")
    with pytest.raises(he.HEError):
        gctx.capture(lambda: gctx.int_weight_table(w, KB, 2, out=buf))
    # the context still works after the refused capture
    t = gctx.int_weight_table(w, KB, 2)
    assert _host(t)[0] == (1 << KB)
