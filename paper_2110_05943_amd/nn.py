"""Warm-start network: ctypes binding of the HIP kernels of include/clb_nn.h
and the encoder-decoder (U-Net) assembled from them.

Argument marshalling and buffer bookkeeping only: every layer, gradient,
loss and optimizer step runs in the HIP library.  PyTorch provides device
memory (tensors used as raw buffers) and the stream.

The network maps a 16-channel input (porosity map, normalised dimensionless
groups, coordinates; clb_nn_features) on an h x w grid to 16 output channels
of which the first three are the predicted steady u / u_c, v / u_c and T - 1/2
of a cavity.  Architecture: five levels of widths 16, 32, 64, 128, 256; two
3x3 convolutions with leaky ReLU (slope 1/8) per level; 2x2 average pooling
down, nearest 2x upsampling and concatenation with the encoder output of the
level on the way up; a final 3x3 convolution without activation (FP32
output).  Mixed precision: bfloat16 activations and gradients, FP32 master
weights, gradients and AdamW moments.
"""
import ctypes as C

import numpy as np

from . import _binding as B

SLOPE = 0.125
NN_EXPORTS = (
    "clb_nn_conv3x3", "clb_nn_wgrad_workspace_bytes", "clb_nn_conv3x3_wgrad",
    "clb_nn_weights_bf16", "clb_nn_pool2", "clb_nn_pool2_grad", "clb_nn_up2", "clb_nn_up2_grad",
    "clb_nn_concat", "clb_nn_split", "clb_nn_act_grad", "clb_nn_mse_workspace_bytes",
    "clb_nn_mse", "clb_nn_adamw", "clb_nn_features", "clb_nn_gather",
    "clb_nn_wgrad_static_max_bytes", "clb_nn_conv3x3_wgrad_static", "clb_nn_conv3x3_cat",
    "clb_nn_conv3x3_split", "clb_nn_conv3x3_wgrad_cat", "clb_nn_weights_bf16_layers",
    "clb_nn_conv3x3_wgrad_parts", "clb_nn_conv3x3_wgrad_cat_parts", "clb_nn_wgrad_reduce_layers",
    "clb_nn_conv3x3_act_grad", "clb_nn_pool2_grad_act", "clb_nn_up2_grad_act",
    "clb_nn_adamw_layers",
)

_ready = False


def lib():
    global _ready
    L = B._lib()
    if not _ready:
        vp, i32, i64, f32, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
        st, sz = C.c_int, C.POINTER(C.c_size_t)
        sig = {
            "clb_nn_conv3x3": [vp, i32, i32, i32, i32, vp, vp, i32, i32, f32, vp, i32, vp],
            "clb_nn_wgrad_workspace_bytes": [i32, i32, i32, i32, i32, sz],
            "clb_nn_conv3x3_wgrad": [vp, vp, i32, i32, i32, i32, i32, vp, vp, vp, C.c_size_t, vp],
            "clb_nn_conv3x3_wgrad_static": [vp, vp, i32, i32, i32, i32, i32, vp, vp, vp],
            "clb_nn_conv3x3_cat": [vp, i32, i32, vp, i32, i32, i32, i32, vp, vp, i32, i32, f32,
                                   vp, i32, vp],
            "clb_nn_conv3x3_split": [vp, i32, i32, i32, i32, vp, i32, i32, vp, vp, vp],
            "clb_nn_conv3x3_wgrad_cat": [vp, vp, i32, i32, vp, i32, i32, i32, i32, i32, vp, vp,
                                         vp, C.c_size_t, vp],
            "clb_nn_weights_bf16": [vp, i32, i32, vp, vp, vp],
            "clb_nn_weights_bf16_layers": [vp, i32, vp, vp, vp, vp, vp, vp],
            "clb_nn_conv3x3_wgrad_parts": [vp, vp, i32, i32, i32, i32, i32, i32, vp, C.c_size_t,
                                           C.POINTER(C.c_int32), vp],
            "clb_nn_conv3x3_wgrad_cat_parts": [vp, vp, i32, i32, vp, i32, i32, i32, i32, i32, i32,
                                               vp, C.c_size_t, C.POINTER(C.c_int32), vp],
            "clb_nn_wgrad_reduce_layers": [i32, vp, vp, vp, vp, vp, vp, vp],
            "clb_nn_conv3x3_act_grad": [vp, i32, i32, i32, i32, vp, i32, vp, f32, vp, vp],
            "clb_nn_pool2_grad_act": [vp, i32, i32, i32, i32, vp, vp, f32, vp, vp],
            "clb_nn_up2_grad_act": [vp, i32, i32, i32, i32, vp, f32, vp, vp],
            "clb_nn_pool2": [vp, i32, i32, i32, i32, vp, vp],
            "clb_nn_pool2_grad": [vp, i32, i32, i32, i32, vp, vp],
            "clb_nn_up2": [vp, i32, i32, i32, i32, vp, vp],
            "clb_nn_up2_grad": [vp, i32, i32, i32, i32, vp, vp],
            "clb_nn_concat": [vp, i32, vp, i32, i64, vp, vp],
            "clb_nn_split": [vp, i32, i32, i64, vp, vp, vp],
            "clb_nn_act_grad": [vp, vp, vp, i64, f32, vp, vp],
            "clb_nn_mse_workspace_bytes": [i64, sz],
            "clb_nn_mse": [vp, i32, vp, i32, i64, vp, vp, vp, C.c_size_t, vp],
            "clb_nn_adamw": [vp, vp, vp, vp, i64, f32, f32, f32, f32, f32, i32, vp],
            "clb_nn_adamw_layers": [vp, vp, vp, vp, i64, f32, f32, f32, f32, f32, i32, i32, vp,
                                    vp, vp, vp, vp, vp],
            "clb_nn_features": [vp, vp, i32, vp, i32, i32, i32, vp, vp],
            "clb_nn_gather": [vp, i32, vp, i32, i64, vp, vp],
            "clb_set_state_device": [vp, i32, vp, i64, f64, f64],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.restype = st
            fn.argtypes = args
        L.clb_nn_wgrad_static_max_bytes.restype = C.c_size_t
        L.clb_nn_wgrad_static_max_bytes.argtypes = []
        _ready = True
    return L


def call(name, *args):
    B._check(getattr(lib(), name)(*args), name)


def ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def graph(levels=5, base=16, cout=16):
    """Steps of the encoder-decoder; step i writes tensor i + 1 (tensor 0 is
    the input): dicts with op in {conv, pool, up, cat}, input tensor ids, and
    for convolutions the index k, the activation flag and the output width."""
    steps, skips = [], []
    cur, k = 0, 0
    for lv in range(levels):
        if lv:
            steps.append(dict(op="pool", ins=[cur]))
            cur = len(steps)
        for _ in range(2):
            steps.append(dict(op="conv", ins=[cur], k=k, act=True, out=base << lv))
            cur, k = len(steps), k + 1
        skips.append(cur)
    for lv in range(levels - 2, -1, -1):
        steps.append(dict(op="up", ins=[cur]))
        steps.append(dict(op="cat", ins=[len(steps), skips[lv]]))
        cur = len(steps)
        for _ in range(2):
            steps.append(dict(op="conv", ins=[cur], k=k, act=True, out=base << lv))
            cur, k = len(steps), k + 1
    steps.append(dict(op="conv", ins=[cur], k=k, act=False, out=cout))
    return steps


class UNet:
    """The encoder-decoder on one device.  Parameters live in one flat FP32
    tensor (per convolution: weights (out, 9, in), then bias (out,)), with
    gradients and AdamW moments of the same layout."""

    def __init__(self, levels=5, base=16, cin=16, cout=16, device="cuda:0", seed=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the warm-start network needs a ROCm GPU; none is visible")
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.levels, self.base, self.cin, self.cout = levels, base, cin, cout
        self.steps = graph(levels, base, cout)
        # channel count and downsampling level of every tensor
        self.ch, self.lv = [cin], [0]
        self.convs = []
        for st in self.steps:
            a = st["ins"][0]
            if st["op"] == "pool":
                self.ch.append(self.ch[a])
                self.lv.append(self.lv[a] + 1)
            elif st["op"] == "up":
                self.ch.append(self.ch[a])
                self.lv.append(self.lv[a] - 1)
            elif st["op"] == "cat":
                self.ch.append(self.ch[a] + self.ch[st["ins"][1]])
                self.lv.append(self.lv[a])
            else:
                self.convs.append((st["out"], self.ch[a]))
                self.ch.append(st["out"])
                self.lv.append(self.lv[a])
        # A decoder convolution reads [up(deep), skip] through the fused
        # gather: fused[i] = (deep, up tensor, skip) for such a convolution
        # step i; the up and cat steps it absorbs are not computed (virtual).
        self.fused, self.virtual = {}, set()
        for i, st in enumerate(self.steps):
            if st["op"] != "conv":
                continue
            a = st["ins"][0]
            cat = self.steps[a - 1] if a > 0 else None
            if cat and cat["op"] == "cat" and self.steps[cat["ins"][0] - 1]["op"] == "up":
                t_up, t_skip = cat["ins"]
                self.fused[i] = (self.steps[t_up - 1]["ins"][0], t_up, t_skip)
                self.virtual |= {a - 1, t_up - 1}
        # gradient contributions each tensor receives in the backward pass (a
        # virtual cat step passes none: its convolution writes both parts),
        # and whether it is the output of a leaky ReLU
        self.expect = [0] * len(self.ch)
        self.expect[-1] = 1  # the loss
        for i, st in enumerate(self.steps):
            if st["op"] == "conv":
                if i in self.fused:
                    _, t_up, skip = self.fused[i]
                    self.expect[t_up] += 1
                    self.expect[skip] += 1
                elif st["ins"][0] > 0:
                    self.expect[st["ins"][0]] += 1
            elif st["op"] in ("pool", "up"):
                self.expect[st["ins"][0]] += 1
            elif i not in self.virtual:
                for a in st["ins"]:
                    self.expect[a] += 1
        self.activated = [t > 0 and self.steps[t - 1]["op"] == "conv" and self.steps[t - 1]["act"]
                          for t in range(len(self.ch))]
        self.offsets = []
        n = 0
        for o, c in self.convs:
            self.offsets.append((n, n + o * 9 * c))
            n += o * 9 * c + o
        self.nparams = n
        f32 = dict(dtype=torch.float32, device=self.device)
        self.p = torch.zeros(n, **f32)
        self.g = torch.zeros(n, **f32)
        self.m = torch.zeros(n, **f32)
        self.v = torch.zeros(n, **f32)
        # bfloat16 copies of the weights (forward and input-gradient layouts)
        # at the parameters' offsets, refreshed in one launch
        self.wf_flat = torch.zeros(n, dtype=torch.bfloat16, device=self.device)
        self.wb_flat = torch.zeros(n, dtype=torch.bfloat16, device=self.device)
        self.wf = [self.wf_flat[w0:b0] for w0, b0 in self.offsets]
        self.wb = [self.wb_flat[w0:b0] for w0, b0 in self.offsets]
        self._layer_tab = (np.array([o for o, _ in self.convs], dtype=np.int32),
                           np.array([c for _, c in self.convs], dtype=np.int32),
                           np.array([w0 for w0, _ in self.offsets], dtype=np.int64))
        self.t = 0
        self.set_params(self.init_params(seed))
        self._shape = None

    # ------------------------------------------------------------ parameters
    def init_params(self, seed):
        """He-normal weights for the leaky ReLU, zero biases (host, seeded)."""
        r = np.random.Generator(np.random.PCG64(seed))
        flat = np.zeros(self.nparams, dtype=np.float32)
        for (o, c), (w0, b0) in zip(self.convs, self.offsets):
            std = np.sqrt(2.0 / (1.0 + SLOPE ** 2) / (9 * c))
            flat[w0:b0] = r.standard_normal(o * 9 * c) * std
        return flat

    def set_params(self, flat):
        self.p.copy_(self.torch.from_numpy(np.ascontiguousarray(flat, dtype=np.float32)))
        self._refresh_bf16()

    def get_params(self):
        return self.p.cpu().numpy()

    def param_list(self):
        """[(w (out, 9, in), b (out,))] as FP32 numpy arrays."""
        flat = self.get_params()
        out = []
        for (o, c), (w0, b0) in zip(self.convs, self.offsets):
            out.append((flat[w0:b0].reshape(o, 9, c).copy(), flat[b0:b0 + o].copy()))
        return out

    def grad_list(self):
        flat = self.g.cpu().numpy()
        return [(flat[w0:b0].reshape(o, 9, c).copy(), flat[b0:b0 + o].copy())
                for (o, c), (w0, b0) in zip(self.convs, self.offsets)]

    def _refresh_bf16(self):
        co, ci, off = self._layer_tab
        call("clb_nn_weights_bf16_layers", ptr(self.p), len(self.convs),
             co.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
             off.ctypes.data_as(C.c_void_p), ptr(self.wf_flat), ptr(self.wb_flat),
             C.c_void_p(self.stream.cuda_stream))

    # --------------------------------------------------------------- buffers
    def _buffers(self, batch, h, w):
        if self._shape == (batch, h, w):
            return
        torch = self.torch
        if h % (1 << (self.levels - 1)) or w % (1 << (self.levels - 1)):
            raise ValueError("image sides must be multiples of %d" % (1 << (self.levels - 1)))
        bf = dict(dtype=torch.bfloat16, device=self.device)
        self.vals, self.grads_t, self.gtmp = [], [], []
        for t, (c, lv) in enumerate(zip(self.ch, self.lv)):
            n = batch * (h >> lv) * (w >> lv) * c
            last = t == len(self.ch) - 1
            if t > 0 and t - 1 in self.virtual:
                self.vals.append(None)  # never formed
                continue
            self.vals.append(torch.empty(n, dtype=torch.float32, device=self.device)
                             if last else torch.empty(n, **bf))
        # gradient storage: per tensor up to two contributions, plus the
        # gradient through the activation
        self.gin = [[None, None] for _ in self.ch]
        self.dz = [None] * len(self.ch)
        for t, (c, lv) in enumerate(zip(self.ch, self.lv)):
            n = batch * (h >> lv) * (w >> lv) * c
            if t > 0 and self.steps[t - 1]["op"] == "cat" and t - 1 in self.virtual:
                continue  # its gradient goes straight to its two parts
            self.gin[t] = [torch.empty(n, **bf), torch.empty(n, **bf)]
            self.dz[t] = torch.empty(n, **bf)
        # one workspace slice per convolution for the weight-gradient partial
        # sums, which one launch adds after the backward pass
        self.ws_off, total = [0] * len(self.convs), 0
        for st in self.steps:
            if st["op"] == "conv":
                a = st["ins"][0]
                nb = C.c_size_t()
                call("clb_nn_wgrad_workspace_bytes", batch, h >> self.lv[a], w >> self.lv[a],
                     self.ch[a], st["out"], C.byref(nb))
                self.ws_off[st["k"]] = total
                total += (nb.value + 255) // 256 * 256
        self.ws_parts = torch.empty(total, dtype=torch.uint8, device=self.device)
        self.ws_bytes = [0] * len(self.convs)
        for k in range(len(self.convs)):
            end = self.ws_off[k + 1] if k + 1 < len(self.convs) else total
            self.ws_bytes[k] = end - self.ws_off[k]
        nb = C.c_size_t()
        call("clb_nn_mse_workspace_bytes", batch * h * w, C.byref(nb))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self.loss_d = torch.zeros(1, dtype=torch.float64, device=self.device)
        self._shape = (batch, h, w)

    # --------------------------------------------------------------- forward
    def forward(self, x, batch, h, w):
        """x: bfloat16 tensor (batch, h, w, cin).  Returns the FP32 output
        tensor (batch, h, w, cout), owned by the network (overwritten by the
        next call)."""
        self._buffers(batch, h, w)
        s = C.c_void_p(self.stream.cuda_stream)
        vals = self.vals
        vals[0] = x
        for i, st in enumerate(self.steps):
            t, a = i + 1, st["ins"][0]
            ha, wa = h >> self.lv[a], w >> self.lv[a]
            if i in self.virtual:
                continue
            if st["op"] == "conv" and i in self.fused:
                k = st["k"]
                w0, b0 = self.offsets[k]
                deep, t_up, skip = self.fused[i]
                call("clb_nn_conv3x3_cat", ptr(vals[deep]), self.ch[deep], 1, ptr(vals[skip]),
                     self.ch[skip], batch, ha, wa, ptr(self.wf[k]),
                     C.c_void_p(self.p.data_ptr() + 4 * b0), st["out"], 1 if st["act"] else 0,
                     SLOPE, ptr(vals[t]), 0 if st["act"] else 1, s)
            elif st["op"] == "conv":
                k = st["k"]
                w0, b0 = self.offsets[k]
                call("clb_nn_conv3x3", ptr(vals[a]), batch, ha, wa, self.ch[a], ptr(self.wf[k]),
                     C.c_void_p(self.p.data_ptr() + 4 * b0), st["out"], 1 if st["act"] else 0,
                     SLOPE, ptr(vals[t]), 0 if st["act"] else 1, s)
            elif st["op"] == "pool":
                call("clb_nn_pool2", ptr(vals[a]), batch, ha, wa, self.ch[a], ptr(vals[t]), s)
            elif st["op"] == "up":
                call("clb_nn_up2", ptr(vals[a]), batch, ha, wa, self.ch[a], ptr(vals[t]), s)
            else:
                b_ = st["ins"][1]
                call("clb_nn_concat", ptr(vals[a]), self.ch[a], ptr(vals[b_]), self.ch[b_],
                     batch * ha * wa, ptr(vals[t]), s)
        return vals[-1]

    # -------------------------------------------------------------- backward
    def backward(self, target, nch, batch, h, w):
        """Mean-squared error of the first nch output channels against target
        (FP32 tensor (batch, h, w, nch)) after forward(); fills the gradient
        tensor self.g and returns the loss as a device FP64 tensor."""
        s = C.c_void_p(self.stream.cuda_stream)
        vals, T = self.vals, len(self.ch) - 1
        ncontrib = [0] * len(self.ch)
        call("clb_nn_mse", ptr(vals[T]), self.ch[T], ptr(target), nch, batch * h * w,
             ptr(self.gin[T][0]), ptr(self.loss_d), ptr(self.ws), self.ws.numel(), s)
        ncontrib[T] = 1

        def contrib(t):
            buf = self.gin[t][ncontrib[t]]
            ncontrib[t] += 1
            return buf

        def completes(t, single=False):
            """This contribution completes the gradient of t, a leaky ReLU
            output: the producer then writes dz[t] itself."""
            return (self.activated[t] and ncontrib[t] + 1 == self.expect[t]
                    and (self.expect[t] == 1 or not single))

        done = [False] * len(self.ch)
        nsplit = [C.c_int32(0) for _ in self.convs]

        for i in range(len(self.steps) - 1, -1, -1):
            st = self.steps[i]
            t, a = i + 1, st["ins"][0]
            if ncontrib[t] == 0:
                continue
            g0 = self.gin[t][0]
            g1 = self.gin[t][1] if ncontrib[t] == 2 else None
            ht, wt = h >> self.lv[t], w >> self.lv[t]
            ha, wa = h >> self.lv[a], w >> self.lv[a]
            if st["op"] == "conv":
                k = st["k"]
                if st["act"] and done[t]:
                    dz = self.dz[t]
                elif st["act"]:
                    call("clb_nn_act_grad", ptr(g0), ptr(g1), ptr(vals[t]),
                         batch * ht * wt * self.ch[t], SLOPE, ptr(self.dz[t]), s)
                    dz = self.dz[t]
                else:
                    dz = g0
                ws_k = C.c_void_p(self.ws_parts.data_ptr() + self.ws_off[k])
                if i in self.fused:
                    deep, t_up, skip = self.fused[i]
                    call("clb_nn_conv3x3_wgrad_cat_parts", ptr(dz), ptr(vals[deep]), self.ch[deep],
                         1, ptr(vals[skip]), self.ch[skip], batch, ha, wa, st["out"], 1, ws_k,
                         self.ws_bytes[k], C.byref(nsplit[k]), s)
                    # input gradient written straight to its two parts
                    call("clb_nn_conv3x3_split", ptr(dz), batch, ha, wa, st["out"],
                         ptr(self.wb[k]), self.ch[a], self.ch[t_up], ptr(contrib(t_up)),
                         ptr(contrib(skip)), s)
                    continue
                call("clb_nn_conv3x3_wgrad_parts", ptr(dz), ptr(vals[a]), batch, ha, wa,
                     self.ch[a], st["out"], 1, ws_k, self.ws_bytes[k], C.byref(nsplit[k]), s)
                if a > 0 and completes(a, single=True):
                    call("clb_nn_conv3x3_act_grad", ptr(dz), batch, ha, wa, st["out"],
                         ptr(self.wb[k]), self.ch[a], ptr(vals[a]), SLOPE, ptr(self.dz[a]), s)
                    ncontrib[a] += 1
                    done[a] = True
                elif a > 0:
                    call("clb_nn_conv3x3", ptr(dz), batch, ha, wa, st["out"], ptr(self.wb[k]),
                         None, self.ch[a], 0, 0.0, ptr(contrib(a)), 0, s)
            elif st["op"] == "pool" and completes(a) and self.ch[a] % 8 == 0:
                add = self.gin[a][0] if self.expect[a] == 2 else None
                call("clb_nn_pool2_grad_act", ptr(g0), batch, ha, wa, self.ch[a], ptr(add),
                     ptr(vals[a]), SLOPE, ptr(self.dz[a]), s)
                ncontrib[a] += 1
                done[a] = True
            elif st["op"] == "pool":
                call("clb_nn_pool2_grad", ptr(g0), batch, ha, wa, self.ch[a], ptr(contrib(a)), s)
            elif st["op"] == "up" and completes(a, single=True) and self.ch[a] % 8 == 0:
                call("clb_nn_up2_grad_act", ptr(g0), batch, ha, wa, self.ch[a], ptr(vals[a]),
                     SLOPE, ptr(self.dz[a]), s)
                ncontrib[a] += 1
                done[a] = True
            elif st["op"] == "up":
                call("clb_nn_up2_grad", ptr(g0), batch, ha, wa, self.ch[a], ptr(contrib(a)), s)
            else:
                b_ = st["ins"][1]
                call("clb_nn_split", ptr(g0), self.ch[a], self.ch[b_], batch * ha * wa,
                     ptr(contrib(a)), ptr(contrib(b_)), s)
        # the weight and bias gradients of every convolution in one launch
        ks = [k for k in range(len(self.convs)) if nsplit[k].value > 0]
        VP = C.c_void_p * len(ks)
        I32 = C.c_int32 * len(ks)
        parts = VP(*[self.ws_parts.data_ptr() + self.ws_off[k] for k in ks])
        dw = VP(*[self.g.data_ptr() + 4 * self.offsets[k][0] for k in ks])
        db = VP(*[self.g.data_ptr() + 4 * self.offsets[k][1] for k in ks])
        call("clb_nn_wgrad_reduce_layers", len(ks), parts, I32(*[nsplit[k].value for k in ks]),
             I32(*[self.convs[k][0] for k in ks]), I32(*[self.convs[k][1] for k in ks]), dw, db,
             s)
        return self.loss_d

    def adamw(self, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
        """One AdamW step on the flat parameters, refreshing the bfloat16
        weight copies in the same launch."""
        self.t += 1
        co, ci, off = self._layer_tab
        call("clb_nn_adamw_layers", ptr(self.p), ptr(self.g), ptr(self.m), ptr(self.v),
             self.nparams, lr, b1, b2, eps, wd, self.t, len(self.convs),
             co.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
             off.ctypes.data_as(C.c_void_p), ptr(self.wf_flat), ptr(self.wb_flat),
             C.c_void_p(self.stream.cuda_stream))
