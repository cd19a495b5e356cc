"""The weight gradient without a workspace (clb_nn_conv3x3_wgrad_static,
for callers that cannot allocate device memory) against the workspace entry
point clb_nn_conv3x3_wgrad and the FP64 oracle: two calls in a row on the
library's per-GPU scratch, the second smaller, each bit-identical to the
workspace call and within the oracle bound."""
import ctypes as C
import sys

import numpy as np
import pytest

from oracle import nn_oracle as N

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_static_scratch_wgrad_matches_workspace_call():
    import torch
    assert torch.cuda.is_available(), "needs the MI355X"
    from paper_2110_05943_amd import nn
    nn.lib()
    r = np.random.Generator(np.random.PCG64(4242))
    # the larger shape first (a 32 -> 64 layer), then a smaller one: the second
    # call must not see the first call's partial sums
    for Bn, H, W, ci, co in ((4, 40, 24, 32, 64), (2, 12, 20, 16, 16)):
        log("static wgrad batch %d %dx%d cin %d cout %d" % (Bn, H, W, ci, co))
        x = N.round_bf16(r.standard_normal((Bn, H, W, ci)))
        dy = N.round_bf16(r.standard_normal((Bn, H, W, co)))
        tx = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).cuda()
        tdy = torch.tensor(dy.astype(np.float32)).to(torch.bfloat16).cuda()
        nb = C.c_size_t()
        nn.call("clb_nn_wgrad_workspace_bytes", Bn, H, W, ci, co, C.byref(nb))
        assert nb.value <= nn.lib().clb_nn_wgrad_static_max_bytes()
        ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        gw_ws = torch.zeros(co * 9 * ci, dtype=torch.float32, device="cuda")
        gb_ws = torch.zeros(co, dtype=torch.float32, device="cuda")
        gw_st = torch.full((co * 9 * ci,), float("nan"), dtype=torch.float32, device="cuda")
        gb_st = torch.full((co,), float("nan"), dtype=torch.float32, device="cuda")
        nn.call("clb_nn_conv3x3_wgrad", nn.ptr(tdy), nn.ptr(tx), Bn, H, W, ci, co, nn.ptr(gw_ws),
                nn.ptr(gb_ws), nn.ptr(ws), nb.value, None)
        nn.call("clb_nn_conv3x3_wgrad_static", nn.ptr(tdy), nn.ptr(tx), Bn, H, W, ci, co,
                nn.ptr(gw_st), nn.ptr(gb_st), None)
        torch.cuda.synchronize()
        assert torch.equal(gw_ws, gw_st) and torch.equal(gb_ws, gb_st)
        rw, rb = N.conv3x3_grad_weight(dy, x)
        bw = N.conv3x3_grad_weight(np.abs(dy), np.abs(x))[0] * 1e-5 + 1e-30
        ew = np.abs(gw_st.cpu().numpy().astype(np.float64).reshape(rw.shape) - rw)
        log("  max err / bound %.3f" % (ew / bw).max())
        assert np.all(ew <= bw)
        assert np.allclose(gb_st.cpu().numpy(), rb, rtol=1e-5,
                           atol=1e-5 * np.abs(dy).sum(axis=(0, 1, 2)).max())
