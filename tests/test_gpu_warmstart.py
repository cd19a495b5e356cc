"""GPU: the learned warm start end to end.

- training with the library's own forward, backward and AdamW kernels lowers
  the loss on a fixed batch;
- the committed network, on held-out cavities (the first 24 of the held-out
  draws, seed 1), predicts the steady fields to a few percent and shortens
  the time to steady state against the plain solver started from rest, with
  the same final Nusselt numbers.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2110_05943_amd", "data", "warmstart_unet.npz")


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "needs the MI355X"
    return t


def test_training_lowers_the_loss(torch):
    from paper_2110_05943_amd import nn
    net = nn.UNet(seed=3)
    r = np.random.Generator(np.random.PCG64(8))
    B, n = 4, 32
    x = torch.tensor(r.standard_normal((B, n, n, 16)), dtype=torch.bfloat16, device="cuda")
    tgt = torch.tensor(0.3 * r.standard_normal((B, n, n, 3)), dtype=torch.float32, device="cuda")
    losses = []
    for _ in range(60):
        net.forward(x, B, n, n)
        losses.append(net.backward(tgt, 3, B, n, n).item())
        net.adamw(2e-3)
    log("loss %.4e -> %.4e" % (losses[0], losses[-1]))
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]


def test_trained_network_shortens_time_to_steady_state(torch):
    from paper_2110_05943_amd import inputs
    from paper_2110_05943_amd import warmstart as W
    from paper_2110_05943_amd.train_warmstart import load_weights
    sur = W.Surrogate(n=128)
    meta = load_weights(WEIGHTS, sur.net)
    log("weights: trained on %s cavities, %s epochs" % (meta.get("train"), meta.get("epochs")))
    draws = inputs.warmstart_draws(24, seed=1)
    r = W.evaluate(sur, draws, tol=1e-9, check_every=5000, max_steps=3_000_000, log=log)
    err = np.array(r["pred_rel_l2"])
    sp = np.array([x if x is not None else -1 for x in r["settle_plain"]], dtype=float)
    sw = np.array([x if x is not None else -1 for x in r["settle_warm"]], dtype=float)
    ok = (sp > 0) & (sw > 0)
    dnu = np.abs(np.array(r["nu_warm"]) - np.array(r["nu_plain"]))[ok]
    log("prediction rel-L2 median %.4f max %.4f; %d of %d compared; steps plain %d warm %d "
        "(%.2fx); |dNu| max %.2e; fallback %d"
        % (np.median(err), err.max(), ok.sum(), len(draws), sp[ok].sum(), sw[ok].sum(),
           sp[ok].sum() / sw[ok].sum(), dnu.max(), r["fallback"]))
    assert np.median(err) < 0.03
    assert ok.sum() >= 16
    assert np.all(dnu <= 1e-4)
    assert sw[ok].sum() * 1.15 <= sp[ok].sum()
