"""FP64 CPU oracle of the learned warm start: a convolutional encoder-decoder
(U-Net) that maps a porosity map and the cavity's dimensionless groups to its
steady (u, v, T) fields, trained with mean-squared error and AdamW.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU-baseline
leg, never by the product path.  Shares no code with the GPU library.

Every function is the plain definition in numpy FP64, NHWC layout:
  conv3x3      y[b,i,j,o] = bias[o] + sum_{t,c} w[o,t,c] x[b,i+di_t,j+dj_t,c]
               with taps t = 3 (di + 1) + (dj + 1), di, dj in {-1, 0, 1},
               and x = 0 outside the image (zero padding);
  its two adjoints (gradient with respect to the input and to the weights);
  2x2 average pooling, nearest-neighbour 2x upsampling, channel concatenation;
  leaky ReLU; mean-squared error; the AdamW update (Loshchilov & Hutter,
  decoupled weight decay, bias-corrected moments).
The network functions can round every stored tensor to bfloat16 at the same
points where the GPU kernels store bfloat16 (round to nearest even), so that
both sides take those rounding decisions in the same precision.

Parity pins (tests/test_nn_oracle.py): conv3x3 against scipy's correlate, the
adjoint identities of the gradients, finite differences of the loss, the
closed form of the first AdamW steps.
"""
import numpy as np

TAPS = [(di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)]


def round_bf16(a):
    """Round FP64 values to the nearest bfloat16 value (ties to even), via
    FP32 (both roundings to nearest; FP64 -> FP32 first is exact for the
    values used here, which are FP32 results or already representable)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- layers

def conv3x3(x, w, bias=None):
    """x (B,H,W,C), w (O,9,C), bias (O,) -> (B,H,W,O)."""
    B, H, W, C = x.shape
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((B, H, W, w.shape[0]))
    for t, (di, dj) in enumerate(TAPS):
        y += xp[:, 1 + di:1 + di + H, 1 + dj:1 + dj + W] @ w[:, t, :].T
    if bias is not None:
        y += bias
    return y


def conv3x3_grad_input(dy, w):
    """Gradient of sum(dy * conv3x3(x, w)) with respect to x."""
    B, H, W, _ = dy.shape
    dxp = np.zeros((B, H + 2, W + 2, w.shape[2]))
    for t, (di, dj) in enumerate(TAPS):
        dxp[:, 1 + di:1 + di + H, 1 + dj:1 + dj + W] += dy @ w[:, t, :]
    return dxp[:, 1:-1, 1:-1]


def conv3x3_grad_weight(dy, x):
    """Gradients of sum(dy * conv3x3(x, w, bias)) with respect to w and bias."""
    B, H, W, C = x.shape
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1] = x
    dw = np.zeros((dy.shape[3], 9, C))
    for t, (di, dj) in enumerate(TAPS):
        xs = xp[:, 1 + di:1 + di + H, 1 + dj:1 + dj + W]
        dw[:, t, :] = np.tensordot(dy, xs, axes=([0, 1, 2], [0, 1, 2]))
    return dw, dy.sum(axis=(0, 1, 2))


def leaky(z, slope):
    return np.where(z > 0, z, slope * z)


def leaky_grad(dy, out, slope):
    """Gradient through y = leaky(z) given the output y (same sign as z)."""
    return np.where(out > 0, dy, slope * dy)


def pool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_grad(dy):
    return 0.25 * np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2)


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_grad(dy):
    B, H, W, C = dy.shape
    return dy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def mse(out, target):
    """Mean over all elements of (out - target)^2 and its gradient."""
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adamw_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One AdamW update at step t >= 1: returns the new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v


# ---------------------------------------------------------------- network

def unet_graph(levels=5, base=16, cout=16):
    """The encoder-decoder as a list of steps (op, input ids, conv output
    width); step i produces tensor i + 1 (tensor 0 is the input).  At encoder
    level l (width base * 2^l): two 3x3 convolutions with leaky ReLU, then 2x2
    average pooling into the next level; on the way up: nearest 2x
    upsampling, concatenation [upsampled, encoder output of that level], two
    3x3 convolutions with leaky ReLU of that level's width; a final 3x3
    convolution to `cout` channels without activation.  Convolutions are
    numbered in order of appearance."""
    steps = []
    cur, conv = 0, 0
    skips = []

    def add(op, ins, **kw):
        steps.append(dict(op=op, ins=ins, **kw))
        return len(steps)

    for lv in range(levels):
        if lv > 0:
            cur = add("pool", [cur])
        for _ in range(2):
            cur = add("conv", [cur], k=conv, act=True, out=base << lv)
            conv += 1
        skips.append(cur)
    for lv in range(levels - 2, -1, -1):
        up = add("up", [cur])
        cur = add("cat", [up, skips[lv]])
        for _ in range(2):
            cur = add("conv", [cur], k=conv, act=True, out=base << lv)
            conv += 1
    add("conv", [cur], k=conv, act=False, out=cout)
    return steps


def unet_shapes(cin=16, base=16, levels=5, cout=16):
    """Weight shapes (O, 9, C) of the convolutions of unet_graph, in order."""
    ch = [cin]
    shapes = []
    for st in unet_graph(levels, base, cout):
        a = st["ins"][0]
        if st["op"] in ("pool", "up"):
            ch.append(ch[a])
        elif st["op"] == "cat":
            ch.append(ch[a] + ch[st["ins"][1]])
        else:
            shapes.append((st["out"], 9, ch[a]))
            ch.append(st["out"])
    return shapes


def _forward(graph, params, x, slope, rnd):
    vals = [rnd(x)]
    out = None
    for st in graph:
        a = vals[st["ins"][0]]
        if st["op"] == "pool":
            v = rnd(pool2(a))
        elif st["op"] == "up":
            v = rnd(up2(a))
        elif st["op"] == "cat":
            v = np.concatenate([a, vals[st["ins"][1]]], axis=3)
        else:
            w, b = params[st["k"]]
            z = conv3x3(a, rnd(w), b)
            if st["act"]:
                v = rnd(leaky(z, slope))
            else:
                # the head is stored in FP32 when the storage is rounded
                v = np.asarray(z, dtype=np.float32).astype(np.float64) if rnd is round_bf16 else z
                out = v
        vals.append(v)
    return out, vals


def unet_forward(params, x, levels=5, base=16, slope=0.1, bf16=True):
    """Output of the network (FP32 head values as FP64).  With bf16, every
    stored tensor and the weights are rounded to bfloat16."""
    rnd = round_bf16 if bf16 else (lambda a: a)
    out, _ = _forward(unet_graph(levels, base, params[-1][0].shape[0]), params, x, slope, rnd)
    return out


def unet_loss_grads(params, x, target, levels=5, base=16, slope=0.1, bf16=True):
    """Mean-squared error of the first target.shape[3] output channels and its
    gradients [(dw, db)] for every convolution, by reverse-mode
    differentiation over the steps of unet_graph.  Gradients are stored (and,
    with bf16, rounded) per step: each step's input gradient is rounded when
    stored; the gradient of a tensor with two consumers is their sum; the
    leaky-ReLU factor is applied to that total and rounded once more."""
    rnd = round_bf16 if bf16 else (lambda a: a)
    graph = unet_graph(levels, base, params[-1][0].shape[0])
    out, vals = _forward(graph, params, x, slope, rnd)
    nout = target.shape[3]
    loss, d = mse(out[..., :nout], target)
    dout = np.zeros_like(out)
    dout[..., :nout] = d
    g = [None] * len(vals)  # gradient contributions, summed per tensor
    g[len(vals) - 1] = [rnd(dout)]
    grads = [None] * len(params)
    for i in range(len(graph) - 1, -1, -1):
        st = graph[i]
        t = i + 1
        if g[t] is None:
            continue
        dt = g[t][0] if len(g[t]) == 1 else rnd(sum(g[t]))
        a = st["ins"][0]

        def push(j, v):
            if j > 0:  # no gradient for the network input
                g[j] = (g[j] or []) + [v]

        if st["op"] == "conv":
            if st["act"]:
                dt = rnd(leaky_grad(dt, vals[t], slope))
            w, _ = params[st["k"]]
            grads[st["k"]] = conv3x3_grad_weight(dt, vals[a])
            push(a, rnd(conv3x3_grad_input(dt, rnd(w))))
        elif st["op"] == "pool":
            push(a, rnd(pool2_grad(dt)))
        elif st["op"] == "up":
            push(a, rnd(up2_grad(dt)))
        else:  # cat
            ca = vals[a].shape[3]
            push(a, dt[..., :ca])
            push(st["ins"][1], dt[..., ca:])
    return loss, grads
