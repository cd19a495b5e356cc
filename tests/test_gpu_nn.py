"""GPU parity of the warm-start network kernels (include/clb_nn.h) against the
FP64 oracle (oracle/nn_oracle.py) on seeded inputs.

bfloat16 inputs are exact in both; FP32 results (convolution outputs, weight
gradients) agree to FP32 summation order, bound 1e-5 relative to the sum of
|terms|; bfloat16 results are compared with the oracle's value rounded the
same way (at most one bfloat16 step apart, rarely)."""
import ctypes as C
import sys

import numpy as np
import pytest

from oracle import nn_oracle as N

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nn():
    import torch
    assert torch.cuda.is_available(), "needs the MI355X"
    from paper_2110_05943_amd import nn as m
    m.lib()
    return m


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def dev_bf16(a):
    import torch
    t = torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16)
    assert np.array_equal(t.float().numpy(), np.asarray(a, dtype=np.float32))  # exact
    return t.cuda()


def dev_f32(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float32)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def empty(n, dtype="bf16"):
    import torch
    return torch.zeros(n, dtype=torch.bfloat16 if dtype == "bf16" else torch.float32,
                       device="cuda")


def bf16_steps(a, b):
    """Distance in bfloat16 steps between two bfloat16-representable arrays."""
    ua = np.asarray(a, dtype=np.float32).view(np.int32) >> 16
    ub = np.asarray(b, dtype=np.float32).view(np.int32) >> 16
    return np.abs(ua.astype(np.int64) - ub.astype(np.int64))


def check_bf16(got, ref, what, frac=1e-3, bound=None):
    """bfloat16 results against the FP64 reference: at most one bfloat16 step
    from the rounded reference, and only for a fraction `frac` of the values.
    With `bound` (the reference's own FP32 error bound per value), values
    whose magnitude is within 1024 bounds of zero, where the FP32 sum itself
    may move the result by several bfloat16 steps, are held to
    |got - ref| <= 2^-7 |ref| + bound instead."""
    d = bf16_steps(got, N.round_bf16(ref))
    sel = np.ones(d.shape, bool) if bound is None else np.abs(ref) > 1024 * bound
    log("%s: %d of %d values one bfloat16 step off, max %d (%d near zero)"
        % (what, int((d[sel] > 0).sum()), d.size, int(d[sel].max()), int((~sel).sum())))
    assert d[sel].max() <= 1 and (d[sel] > 0).mean() <= frac
    if bound is not None:
        assert np.all(np.abs(got - ref)[~sel] <= 2.0 ** -7 * np.abs(ref[~sel]) + bound[~sel])


# (batch, h, w, cin, cout).  (1, 255, 259, 32, 48) has over 1024 tiles of 64
# pixels: the convolution takes its pixel-tiled path there (the small shapes
# split the reduction over the waves), with a ragged last tile and a partial
# column tile.  The last two stage bands of whole rows in LDS (at least 256
# bands), the second of them with a partial column tile; the weight gradient
# runs over bands of rows wherever the width is a multiple of 8.
CONV_SHAPES = [(2, 9, 13, 16, 16), (1, 5, 7, 48, 80), (2, 8, 8, 384, 128), (3, 16, 16, 16, 32),
               (1, 255, 259, 32, 48), (4, 128, 128, 16, 16), (16, 64, 64, 32, 48)]


@pytest.mark.parametrize("shape", CONV_SHAPES)
def test_conv3x3_forward_fp32_and_bf16(nn, shape):
    Bn, H, W, ci, co = shape
    r = rng(sum(shape))
    x = N.round_bf16(r.standard_normal((Bn, H, W, ci)))
    w = N.round_bf16(r.standard_normal((co, 9, ci)) / np.sqrt(9 * ci))
    b = r.standard_normal(co).astype(np.float32).astype(np.float64)
    ref = N.conv3x3(x, w, b)
    bound = N.conv3x3(np.abs(x), np.abs(w), np.abs(b)) * 1e-5 + 1e-30
    dx, dw, db = dev_bf16(x), dev_bf16(w), dev_f32(b)
    y32 = empty(ref.size, "f32")
    nn.call("clb_nn_conv3x3", nn.ptr(dx), Bn, H, W, ci, nn.ptr(dw), nn.ptr(db), co, 0, 0.0,
            nn.ptr(y32), 1, None)
    got = host(y32).reshape(ref.shape)
    err = np.abs(got - ref)
    log("conv %s fp32 max err / bound %.3f" % (shape, (err / bound).max()))
    assert np.all(err <= bound)
    y16 = empty(ref.size)
    nn.call("clb_nn_conv3x3", nn.ptr(dx), Bn, H, W, ci, nn.ptr(dw), nn.ptr(db), co, 1,
            nn.SLOPE, nn.ptr(y16), 0, None)
    check_bf16(host(y16).reshape(ref.shape), N.leaky(ref, nn.SLOPE), "conv %s bf16" % (shape,),
               bound=bound)


@pytest.mark.parametrize("shape", CONV_SHAPES)
def test_conv3x3_input_and_weight_gradients(nn, shape):
    Bn, H, W, ci, co = shape
    r = rng(7 + sum(shape))
    x = N.round_bf16(r.standard_normal((Bn, H, W, ci)))
    w32 = (r.standard_normal((co, 9, ci)) / np.sqrt(9 * ci)).astype(np.float32)
    dy = N.round_bf16(r.standard_normal((Bn, H, W, co)))
    wf, wb = empty(w32.size), empty(w32.size)
    tw = dev_f32(w32)
    nn.call("clb_nn_weights_bf16", nn.ptr(tw), co, ci, nn.ptr(wf), nn.ptr(wb), None)
    w = N.round_bf16(w32)
    assert np.array_equal(host(wf).reshape(co, 9, ci), w)
    assert np.array_equal(host(wb).reshape(ci, 9, co), w[:, ::-1, :].transpose(2, 1, 0))
    # input gradient: the forward kernel with the reversed-tap weights
    ddy = dev_bf16(dy)
    gx = empty(x.size, "f32")
    nn.call("clb_nn_conv3x3", nn.ptr(ddy), Bn, H, W, co, nn.ptr(wb), None, ci, 0, 0.0,
            nn.ptr(gx), 1, None)
    ref = N.conv3x3_grad_input(dy, w)
    bound = N.conv3x3_grad_input(np.abs(dy), np.abs(w)) * 1e-5 + 1e-30
    assert np.all(np.abs(host(gx).reshape(ref.shape) - ref) <= bound)
    # weight and bias gradients
    nb = C.c_size_t()
    nn.call("clb_nn_wgrad_workspace_bytes", Bn, H, W, ci, co, C.byref(nb))
    import torch
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    gw, gb = empty(w.size, "f32"), empty(co, "f32")
    tx = dev_bf16(x)
    nn.call("clb_nn_conv3x3_wgrad", nn.ptr(ddy), nn.ptr(tx), Bn, H, W, ci, co,
            nn.ptr(gw), nn.ptr(gb), nn.ptr(ws), nb.value, None)
    rw, rb = N.conv3x3_grad_weight(dy, x)
    bw = N.conv3x3_grad_weight(np.abs(dy), np.abs(x))[0] * 1e-5 + 1e-30
    ew = np.abs(host(gw).reshape(rw.shape) - rw)
    log("wgrad %s max err / bound %.3f" % (shape, (ew / bw).max()))
    assert np.all(ew <= bw)
    assert np.allclose(host(gb), rb, rtol=1e-5, atol=1e-5 * np.abs(dy).sum(axis=(0, 1, 2)).max())
    # deterministic: a second call gives identical bits
    gw2 = empty(w.size, "f32")
    nn.call("clb_nn_conv3x3_wgrad", nn.ptr(ddy), nn.ptr(tx), Bn, H, W, ci, co,
            nn.ptr(gw2), None, nn.ptr(ws), nb.value, None)
    assert torch.equal(gw, gw2)


def test_weights_bf16_layers_matches_per_layer_calls(nn):
    """One launch for the layers of a flat parameter array gives the bits of
    the per-layer conversion and leaves the elements between layers alone."""
    import torch
    r = rng(19)
    layers = [(16, 16), (32, 48), (16, 272)]  # (cout, cin)
    offs, n = [], 0
    for o, c in layers:
        offs.append(n)
        n += o * 9 * c + o + 32  # weights, a bias and a gap
    w32 = dev_f32(r.standard_normal(n).astype(np.float32))
    sentinel = torch.full((n,), 7.0, dtype=torch.bfloat16, device="cuda")
    wf, wb = sentinel.clone(), sentinel.clone()
    co = np.array([o for o, _ in layers], dtype=np.int32)
    ci = np.array([c for _, c in layers], dtype=np.int32)
    off = np.array(offs, dtype=np.int64)
    nn.call("clb_nn_weights_bf16_layers", nn.ptr(w32), len(layers), co.ctypes.data_as(C.c_void_p),
            ci.ctypes.data_as(C.c_void_p), off.ctypes.data_as(C.c_void_p), nn.ptr(wf), nn.ptr(wb),
            None)
    torch.cuda.synchronize()
    covered = torch.zeros(n, dtype=torch.bool, device="cuda")
    for (o, c), w0 in zip(layers, offs):
        m = o * 9 * c
        rf, rb = empty(m), empty(m)
        nn.call("clb_nn_weights_bf16", C.c_void_p(w32.data_ptr() + 4 * w0), o, c, nn.ptr(rf),
                nn.ptr(rb), None)
        assert torch.equal(wf[w0:w0 + m].view(torch.int16), rf.view(torch.int16))
        assert torch.equal(wb[w0:w0 + m].view(torch.int16), rb.view(torch.int16))
        covered[w0:w0 + m] = True
    assert torch.equal(wf[~covered], sentinel[~covered])
    assert torch.equal(wb[~covered], sentinel[~covered])
    bad = np.array([0], dtype=np.int32)
    assert nn.lib().clb_nn_weights_bf16_layers(nn.ptr(w32), 1, bad.ctypes.data_as(C.c_void_p),
                                               ci.ctypes.data_as(C.c_void_p),
                                               off.ctypes.data_as(C.c_void_p), nn.ptr(wf),
                                               nn.ptr(wb), None) != 0


def test_wgrad_parts_and_one_reduction_match_wgrad(nn):
    """clb_nn_conv3x3_wgrad_parts (row-band and tiled kernels) and
    clb_nn_conv3x3_wgrad_cat_parts, added for all layers by one
    clb_nn_wgrad_reduce_layers, give the bits of clb_nn_conv3x3_wgrad and
    clb_nn_conv3x3_wgrad_cat."""
    import torch
    r = rng(23)
    # (batch, h, w, cin or (ca, cb), cout, bias)
    layers = [(2, 16, 16, 16, 32, True), (1, 9, 13, 32, 16, False), (2, 16, 16, (32, 16), 16, True)]
    parts, ns, co, ci, dws, dbs, refs, keep = [], [], [], [], [], [], [], []
    for Bn, H, W, cin, cout, with_b in layers:
        cat = isinstance(cin, tuple)
        ct = sum(cin) if cat else cin
        dy = dev_bf16(N.round_bf16(r.standard_normal((Bn, H, W, cout))))
        nb = C.c_size_t()
        nn.call("clb_nn_wgrad_workspace_bytes", Bn, H, W, ct, cout, C.byref(nb))
        ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        ws_ref = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        gw, gb = empty(cout * 9 * ct, "f32"), empty(cout, "f32") if with_b else None
        rw, rb = empty(cout * 9 * ct, "f32"), empty(cout, "f32") if with_b else None
        n = C.c_int32(0)
        if cat:
            ca, cb = cin
            a = dev_bf16(N.round_bf16(r.standard_normal((Bn, H // 2, W // 2, ca))))
            b = dev_bf16(N.round_bf16(r.standard_normal((Bn, H, W, cb))))
            nn.call("clb_nn_conv3x3_wgrad_cat", nn.ptr(dy), nn.ptr(a), ca, 1, nn.ptr(b), cb, Bn, H,
                    W, cout, nn.ptr(rw), nn.ptr(rb), nn.ptr(ws_ref), nb.value, None)
            nn.call("clb_nn_conv3x3_wgrad_cat_parts", nn.ptr(dy), nn.ptr(a), ca, 1, nn.ptr(b), cb,
                    Bn, H, W, cout, int(with_b), nn.ptr(ws), nb.value, C.byref(n), None)
            keep += [a, b]
        else:
            x = dev_bf16(N.round_bf16(r.standard_normal((Bn, H, W, cin))))
            nn.call("clb_nn_conv3x3_wgrad", nn.ptr(dy), nn.ptr(x), Bn, H, W, cin, cout,
                    nn.ptr(rw), nn.ptr(rb), nn.ptr(ws_ref), nb.value, None)
            nn.call("clb_nn_conv3x3_wgrad_parts", nn.ptr(dy), nn.ptr(x), Bn, H, W, cin, cout,
                    int(with_b), nn.ptr(ws), nb.value, C.byref(n), None)
            keep.append(x)
        assert n.value >= 1
        keep += [dy, ws, ws_ref]
        parts.append(ws.data_ptr())
        ns.append(n.value)
        co.append(cout)
        ci.append(ct)
        dws.append(gw)
        dbs.append(gb)
        refs.append((rw, rb))
    L = len(layers)
    VP, I32 = C.c_void_p * L, C.c_int32 * L
    nn.call("clb_nn_wgrad_reduce_layers", L, VP(*parts), I32(*ns), I32(*co), I32(*ci),
            VP(*[t.data_ptr() for t in dws]),
            VP(*[t.data_ptr() if t is not None else None for t in dbs]), None)
    torch.cuda.synchronize()
    for gw, gb, (rw, rb) in zip(dws, dbs, refs):
        assert torch.equal(gw, rw)
        assert (gb is None) == (rb is None) and (gb is None or torch.equal(gb, rb))


def test_fused_activation_gradients_match_unfused(nn):
    """clb_nn_conv3x3_act_grad, clb_nn_pool2_grad_act (with and without a
    second contribution) and clb_nn_up2_grad_act give the bits of the
    unfused call followed by clb_nn_act_grad."""
    import torch
    r = rng(29)
    Bn, H, W, c = 2, 16, 24, 32

    def bf(shape):
        return dev_bf16(N.round_bf16(r.standard_normal(shape)))

    def act_ref(g0, g1, y):
        out = empty(y.numel())
        nn.call("clb_nn_act_grad", nn.ptr(g0), nn.ptr(g1), nn.ptr(y), y.numel(), nn.SLOPE,
                nn.ptr(out), None)
        return out

    # input gradient of a convolution (cout = c) from dy with 16 channels
    dy = bf((Bn, H, W, 16))
    w = bf((c, 9, 16)).reshape(-1)  # the input-gradient weights, layout (c, 9, 16)
    y = bf((Bn, H, W, c))
    g = empty(Bn * H * W * c)
    nn.call("clb_nn_conv3x3", nn.ptr(dy), Bn, H, W, 16, nn.ptr(w), None, c, 0, 0.0, nn.ptr(g), 0,
            None)
    ref = act_ref(g, None, y)
    dz = empty(Bn * H * W * c)
    nn.call("clb_nn_conv3x3_act_grad", nn.ptr(dy), Bn, H, W, 16, nn.ptr(w), c, nn.ptr(y),
            nn.SLOPE, nn.ptr(dz), None)
    torch.cuda.synchronize()
    assert torch.equal(dz.view(torch.int16), ref.view(torch.int16))
    # pooling gradient, alone and with another contribution
    dyp = bf((Bn, H // 2, W // 2, c))
    other = bf((Bn, H, W, c))
    gp = empty(Bn * H * W * c)
    nn.call("clb_nn_pool2_grad", nn.ptr(dyp), Bn, H, W, c, nn.ptr(gp), None)
    for add in (None, other):
        ref = act_ref(gp, None, y) if add is None else act_ref(add, gp, y)
        dz = empty(Bn * H * W * c)
        nn.call("clb_nn_pool2_grad_act", nn.ptr(dyp), Bn, H, W, c, nn.ptr(add), nn.ptr(y),
                nn.SLOPE, nn.ptr(dz), None)
        torch.cuda.synchronize()
        assert torch.equal(dz.view(torch.int16), ref.view(torch.int16))
    # upsampling gradient
    yh = bf((Bn, H // 2, W // 2, c))
    gu = empty(Bn * (H // 2) * (W // 2) * c)
    nn.call("clb_nn_up2_grad", nn.ptr(other), Bn, H // 2, W // 2, c, nn.ptr(gu), None)
    ref = act_ref(gu, None, yh)
    dz = empty(gu.numel())
    nn.call("clb_nn_up2_grad_act", nn.ptr(other), Bn, H // 2, W // 2, c, nn.ptr(yh), nn.SLOPE,
            nn.ptr(dz), None)
    torch.cuda.synchronize()
    assert torch.equal(dz.view(torch.int16), ref.view(torch.int16))


def test_adamw_layers_matches_adamw_and_weight_copies(nn):
    """clb_nn_adamw_layers gives the bits of clb_nn_adamw followed by
    clb_nn_weights_bf16_layers, and leaves the bfloat16 elements outside the
    layers' weights alone."""
    import torch
    r = rng(37)
    layers = [(16, 16), (32, 16), (16, 48)]
    offs, n = [], 0
    for o, c in layers:
        offs.append(n)
        n += o * 9 * c + o
    n += 40  # parameters after the last layer
    p0, g = r.standard_normal(n).astype(np.float32), r.standard_normal(n).astype(np.float32)
    m0, v0 = r.standard_normal(n).astype(np.float32), np.abs(r.standard_normal(n)).astype(np.float32)
    co = np.array([o for o, _ in layers], dtype=np.int32)
    ci = np.array([c for _, c in layers], dtype=np.int32)
    off = np.array(offs, dtype=np.int64)
    tab = [t.ctypes.data_as(C.c_void_p) for t in (co, ci, off)]
    a = [dev_f32(x) for x in (p0, g, m0, v0)]
    b = [dev_f32(x) for x in (p0, g, m0, v0)]
    sentinel = torch.full((n,), 3.0, dtype=torch.bfloat16, device="cuda")
    wf_a, wb_a, wf_b, wb_b = (sentinel.clone() for _ in range(4))
    args = (1e-3, 0.9, 0.999, 1e-8, 0.01, 3)
    nn.call("clb_nn_adamw", *[nn.ptr(x) for x in a], n, *args, None)
    nn.call("clb_nn_weights_bf16_layers", nn.ptr(a[0]), len(layers), *tab, nn.ptr(wf_a),
            nn.ptr(wb_a), None)
    nn.call("clb_nn_adamw_layers", *[nn.ptr(x) for x in b], n, *args, len(layers), *tab,
            nn.ptr(wf_b), nn.ptr(wb_b), None)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert torch.equal(wf_a.view(torch.int16), wf_b.view(torch.int16))
    assert torch.equal(wb_a.view(torch.int16), wb_b.view(torch.int16))


def test_elementwise_layers(nn):
    r = rng(11)
    Bn, H, W, Cc = 2, 6, 10, 16
    x = N.round_bf16(r.standard_normal((Bn, H, W, Cc)))
    dx = dev_bf16(x)
    y = empty(x.size // 4)
    nn.call("clb_nn_pool2", nn.ptr(dx), Bn, H, W, Cc, nn.ptr(y), None)
    check_bf16(host(y).reshape(Bn, H // 2, W // 2, Cc), N.pool2(x), "pool2", frac=1e-2)
    dy = N.round_bf16(r.standard_normal((Bn, H // 2, W // 2, Cc)))
    g = empty(x.size)
    tdy = dev_bf16(dy)
    nn.call("clb_nn_pool2_grad", nn.ptr(tdy), Bn, H, W, Cc, nn.ptr(g), None)
    assert np.array_equal(host(g).reshape(x.shape), N.pool2_grad(dy))
    u = empty(x.size * 4)
    nn.call("clb_nn_up2", nn.ptr(dx), Bn, H, W, Cc, nn.ptr(u), None)
    assert np.array_equal(host(u).reshape(Bn, 2 * H, 2 * W, Cc), N.up2(x))
    du = N.round_bf16(r.standard_normal((Bn, 2 * H, 2 * W, Cc)))
    tdu = dev_bf16(du)
    nn.call("clb_nn_up2_grad", nn.ptr(tdu), Bn, H, W, Cc, nn.ptr(g), None)
    check_bf16(host(g).reshape(x.shape), N.up2_grad(du), "up2_grad", frac=1e-2)
    b2 = N.round_bf16(r.standard_normal((Bn, H, W, 32)))
    cat = empty(x.size * 3)
    tb2 = dev_bf16(b2)
    nn.call("clb_nn_concat", nn.ptr(dx), 16, nn.ptr(tb2), 32, Bn * H * W, nn.ptr(cat), None)
    ref = np.concatenate([x, b2], axis=3)
    assert np.array_equal(host(cat).reshape(ref.shape), ref)
    sa, sb = empty(x.size), empty(b2.size)
    nn.call("clb_nn_split", nn.ptr(cat), 16, 32, Bn * H * W, nn.ptr(sa), nn.ptr(sb), None)
    assert np.array_equal(host(sa), x.ravel()) and np.array_equal(host(sb), b2.ravel())
    # activation gradient with one and with two contributions
    out = N.round_bf16(N.leaky(r.standard_normal(x.size), nn.SLOPE))
    g0 = N.round_bf16(r.standard_normal(x.size))
    g1 = N.round_bf16(r.standard_normal(x.size) * 1e-2)
    dz = empty(x.size)
    t0, t1, to = dev_bf16(g0), dev_bf16(g1), dev_bf16(out)
    nn.call("clb_nn_act_grad", nn.ptr(t0), None, nn.ptr(to), x.size, nn.SLOPE, nn.ptr(dz), None)
    assert np.array_equal(host(dz), N.round_bf16(N.leaky_grad(g0, out, nn.SLOPE)))
    nn.call("clb_nn_act_grad", nn.ptr(t0), nn.ptr(t1), nn.ptr(to), x.size, nn.SLOPE, nn.ptr(dz),
            None)
    assert np.array_equal(host(dz), N.round_bf16(N.leaky_grad(N.round_bf16(g0 + g1), out,
                                                              nn.SLOPE)))


def test_mse_adamw_features_gather(nn):
    import torch
    r = rng(12)
    npix, ldo, nch = 1000, 16, 3
    out = r.standard_normal((npix, ldo)).astype(np.float32).astype(np.float64)
    tgt = r.standard_normal((npix, nch)).astype(np.float32).astype(np.float64)
    nb = C.c_size_t()
    nn.call("clb_nn_mse_workspace_bytes", npix, C.byref(nb))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dout = empty(npix * ldo)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    tout, ttgt = dev_f32(out), dev_f32(tgt)
    nn.call("clb_nn_mse", nn.ptr(tout), ldo, nn.ptr(ttgt), nch, npix, nn.ptr(dout), nn.ptr(loss),
            nn.ptr(ws), nb.value, None)
    rl, rg = N.mse(out[:, :nch], tgt)
    assert abs(loss.item() - rl) <= 1e-6 * rl
    g = host(dout).reshape(npix, ldo)
    assert np.all(g[:, nch:] == 0)
    check_bf16(g[:, :nch], rg, "mse grad")
    # AdamW over a few steps
    n = 5000
    p0 = r.standard_normal(n).astype(np.float32)
    p, m, v = dev_f32(p0), empty(n, "f32"), empty(n, "f32")
    rp, rm, rv = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 4):
        gr = r.standard_normal(n).astype(np.float32)
        tg = dev_f32(gr)
        nn.call("clb_nn_adamw", nn.ptr(p), nn.ptr(tg), nn.ptr(m), nn.ptr(v), n, 1e-2,
                0.9, 0.999, 1e-8, 1e-2, t, None)
        torch.cuda.synchronize()
        rp, rm, rv = N.adamw_step(rp, gr.astype(np.float64), rm, rv, t, 1e-2, wd=1e-2)
    assert np.allclose(host(p), rp, rtol=0, atol=1e-6)
    # features and gather
    S, H, W, ng = 5, 8, 16, 4
    eps = r.uniform(0.3, 0.95, (S, H, W)).astype(np.float32)
    groups = r.standard_normal((S, ng)).astype(np.float32)
    idx = np.array([3, 0, 3], dtype=np.int32)
    xf = empty(3 * H * W * 16)
    te, tgr, ti = dev_f32(eps), dev_f32(groups), torch.tensor(idx).cuda()
    nn.call("clb_nn_features", nn.ptr(te), nn.ptr(tgr), ng, nn.ptr(ti), 3, H, W, nn.ptr(xf), None)
    f = host(xf).reshape(3, H, W, 16)
    assert np.array_equal(f[..., 0], N.round_bf16((eps[idx].astype(np.float64) - 0.625) * 5))
    assert np.array_equal(f[1, 2, 3, 1:1 + ng], N.round_bf16(groups[0]))
    assert f[0, 0, 0, ng + 1] == -1.0 and f[0, 0, W - 1, ng + 1] == 1.0
    assert f[0, H - 1, 0, ng + 2] == 1.0 and np.all(f[..., ng + 3:] == 0)
    fields = r.standard_normal((S, H * W, 3)).astype(np.float32)
    tg = empty(3 * H * W * 3, "f32")
    tf = dev_f32(fields)
    nn.call("clb_nn_gather", nn.ptr(tf), 3, nn.ptr(ti), 3, H * W, nn.ptr(tg), None)
    assert np.array_equal(host(tg).reshape(3, H * W, 3), fields[idx])


def test_unet_loss_and_gradients_match_oracle(nn):
    """Three-level network (widths 16, 32, 64) on a batch of two 16 x 16
    inputs: output, loss and every parameter gradient against the oracle's
    reverse pass with the same bfloat16 storage points."""
    import torch
    net = nn.UNet(levels=3, base=16, cin=16, cout=16, seed=3)
    r = rng(13)
    Bn, H, W = 2, 16, 16
    x = N.round_bf16(r.standard_normal((Bn, H, W, 16)))
    tgt = r.standard_normal((Bn, H, W, 3)).astype(np.float32).astype(np.float64)
    params = [(w.astype(np.float64), b.astype(np.float64)) for w, b in net.param_list()]
    tx = dev_bf16(x)
    out = net.forward(tx, Bn, H, W)
    ro = N.unet_forward(params, x, levels=3, base=16, slope=nn.SLOPE)
    eo = np.linalg.norm(host(out).reshape(ro.shape) - ro) / np.linalg.norm(ro)
    ttgt = dev_f32(tgt)
    loss = net.backward(ttgt, 3, Bn, H, W)
    rl, rg = N.unet_loss_grads(params, x, tgt, levels=3, base=16, slope=nn.SLOPE)
    gl = net.grad_list()
    errs = []
    for (gw, gb), (rw, rb) in zip(gl, rg):
        errs.append(max(np.linalg.norm(gw - rw) / np.linalg.norm(rw),
                        np.linalg.norm(gb - rb) / max(np.linalg.norm(rb), 1e-30)))
    log("unet output rel-L2 %.2e, loss gpu %.9f oracle %.9f, worst grad rel-L2 %.2e"
        % (eo, loss.item(), rl, max(errs)))
    assert eo <= 1e-3
    assert abs(loss.item() - rl) <= 1e-3 * rl
    assert max(errs) <= 1e-2
    torch.cuda.synchronize()


# Decoder-level shapes (batch, h, w, ca, cb, cout): the deep tensor a at half
# resolution (ca channels), the skip tensor b at full resolution.  The second
# has over 1024 tiles of 64 pixels (pixel-tiled path with a ragged last tile);
# the first splits the reduction over the waves; the last stages bands of
# whole rows in LDS (the level-0 decoder convolution of the warm-start
# network at batch 4).
CAT_SHAPES = [(2, 8, 12, 32, 16, 16), (2, 96, 64, 32, 32, 32), (1, 16, 16, 128, 64, 64),
              (4, 128, 128, 32, 16, 16)]


@pytest.mark.parametrize("shape", CAT_SHAPES)
def test_fused_decoder_convolution(nn, shape):
    """clb_nn_conv3x3_cat reads [up2(a), b] without forming it: bit-identical
    to clb_nn_up2 + clb_nn_concat + clb_nn_conv3x3, and within the FP32 bound
    of the oracle's convolution of the formed tensor.  Its weight gradient
    (clb_nn_conv3x3_wgrad_cat) and the split input gradient
    (clb_nn_conv3x3_split) match the formed path bit for bit as well."""
    import torch
    Bn, H, W, ca, cb, co = shape
    ci = ca + cb
    r = rng(31 + sum(shape))
    a = N.round_bf16(r.standard_normal((Bn, H // 2, W // 2, ca)))
    b = N.round_bf16(r.standard_normal((Bn, H, W, cb)))
    w = N.round_bf16(r.standard_normal((co, 9, ci)) / np.sqrt(9 * ci))
    bias = r.standard_normal(co).astype(np.float32).astype(np.float64)
    x = np.concatenate([N.up2(a), b], axis=3)
    ref = N.conv3x3(x, w, bias)
    bound = N.conv3x3(np.abs(x), np.abs(w), np.abs(bias)) * 1e-5 + 1e-30
    da, db_, dw, dbias = dev_bf16(a), dev_bf16(b), dev_bf16(w), dev_f32(bias)
    # the formed path
    up = empty(Bn * H * W * ca)
    cat = empty(Bn * H * W * ci)
    nn.call("clb_nn_up2", nn.ptr(da), Bn, H // 2, W // 2, ca, nn.ptr(up), None)
    nn.call("clb_nn_concat", nn.ptr(up), ca, nn.ptr(db_), cb, Bn * H * W, nn.ptr(cat), None)
    for fp32 in (1, 0):
        y_ref = empty(ref.size, "f32" if fp32 else "bf16")
        y = empty(ref.size, "f32" if fp32 else "bf16")
        nn.call("clb_nn_conv3x3", nn.ptr(cat), Bn, H, W, ci, nn.ptr(dw), nn.ptr(dbias), co,
                1 - fp32, nn.SLOPE, nn.ptr(y_ref), fp32, None)
        nn.call("clb_nn_conv3x3_cat", nn.ptr(da), ca, 1, nn.ptr(db_), cb, Bn, H, W, nn.ptr(dw),
                nn.ptr(dbias), co, 1 - fp32, nn.SLOPE, nn.ptr(y), fp32, None)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        if fp32:
            err = np.abs(host(y).reshape(ref.shape) - ref)
            log("fused conv %s fp32 max err / bound %.3f" % (shape, (err / bound).max()))
            assert np.all(err <= bound)
    # weight gradient on the same input
    dy = N.round_bf16(r.standard_normal((Bn, H, W, co)))
    ddy = dev_bf16(dy)
    nb = C.c_size_t()
    nn.call("clb_nn_wgrad_workspace_bytes", Bn, H, W, ci, co, C.byref(nb))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    gw_ref, gb_ref = empty(w.size, "f32"), empty(co, "f32")
    gw, gb = empty(w.size, "f32"), empty(co, "f32")
    nn.call("clb_nn_conv3x3_wgrad", nn.ptr(ddy), nn.ptr(cat), Bn, H, W, ci, co, nn.ptr(gw_ref),
            nn.ptr(gb_ref), nn.ptr(ws), nb.value, None)
    nn.call("clb_nn_conv3x3_wgrad_cat", nn.ptr(ddy), nn.ptr(da), ca, 1, nn.ptr(db_), cb, Bn, H, W,
            co, nn.ptr(gw), nn.ptr(gb), nn.ptr(ws), nb.value, None)
    torch.cuda.synchronize()
    assert torch.equal(gw, gw_ref) and torch.equal(gb, gb_ref)
    rw, _ = N.conv3x3_grad_weight(dy, x)
    bw = N.conv3x3_grad_weight(np.abs(dy), np.abs(x))[0] * 1e-5 + 1e-30
    assert np.all(np.abs(host(gw).reshape(rw.shape) - rw) <= bw)
    # input gradient split into the two parts
    wf, wb = empty(w.size), empty(w.size)
    tw = dev_f32(w)
    nn.call("clb_nn_weights_bf16", nn.ptr(tw), co, ci, nn.ptr(wf), nn.ptr(wb), None)
    gx = empty(x.size)
    nn.call("clb_nn_conv3x3", nn.ptr(ddy), Bn, H, W, co, nn.ptr(wb), None, ci, 0, 0.0,
            nn.ptr(gx), 0, None)
    ga_ref, gb2_ref = empty(Bn * H * W * ca), empty(Bn * H * W * cb)
    nn.call("clb_nn_split", nn.ptr(gx), ca, cb, Bn * H * W, nn.ptr(ga_ref), nn.ptr(gb2_ref), None)
    ga, gb2 = empty(Bn * H * W * ca), empty(Bn * H * W * cb)
    nn.call("clb_nn_conv3x3_split", nn.ptr(ddy), Bn, H, W, co, nn.ptr(wb), ci, ca, nn.ptr(ga),
            nn.ptr(gb2), None)
    torch.cuda.synchronize()
    assert torch.equal(ga, ga_ref) and torch.equal(gb2, gb2_ref)
