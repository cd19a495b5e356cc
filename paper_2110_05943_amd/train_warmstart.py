"""Train the warm-start network on solver-generated steady states.

  python -m paper_2110_05943_amd.train_warmstart --train 4000 --epochs 300 --lr 1e-3 \
      --max-steps 3000000 --out paper_2110_05943_amd/data/warmstart_unet.npz

(the command that wrote the committed weights)

1. Draw `--train` cavities (inputs.warmstart_draws, seed 0): 128^2 nodes,
   Ra log-uniform [1e3, 1e7], mean Da log-uniform [1e-5, 1e-1], Pr in
   {0.71, 1, 7}, sigma uniform [0.8, 1.2], Gaussian-random-field porosity map
   (correlation length 8) with uniform marginal on [0.3, 0.95].
2. Run all of them in one solver context from rest to steady state (relative
   change per step <= --tol over rounds of --check steps, or --max-steps).
3. Train the U-Net (nn.UNet) on (porosity map, groups) -> (u/u_c, v/u_c,
   T - 1/2) with mean-squared error and AdamW, batch 32, cosine decay.
4. Save the weights (bfloat16 bit patterns) and biases (FP32) to --out.
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, flush=True)


def save_weights(path, net, meta):
    flat = net.get_params()
    ws, bs = [], []
    for (o, c), (w0, b0) in zip(net.convs, net.offsets):
        w = flat[w0:b0].astype(np.float32)
        bits = w.view(np.uint32).astype(np.uint64)
        bits = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16).astype(np.uint16)  # nearest even
        ws.append(bits)
        bs.append(flat[b0:b0 + o].astype(np.float32))
    arrays = {"w%02d" % k: w for k, w in enumerate(ws)}
    arrays.update({"b%02d" % k: b for k, b in enumerate(bs)})
    arrays["meta"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, **arrays)


def load_weights(path, net):
    """Weights saved by save_weights into a UNet of the same shape."""
    z = np.load(path, allow_pickle=False)
    flat = np.zeros(net.nparams, dtype=np.float32)
    for k, ((o, c), (w0, b0)) in enumerate(zip(net.convs, net.offsets)):
        bits = z["w%02d" % k].astype(np.uint32) << 16
        flat[w0:b0] = bits.view(np.float32)
        flat[b0:b0 + o] = z["b%02d" % k]
    net.set_params(flat)
    return json.loads(bytes(z["meta"]).decode())


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=4000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--check", type=int, default=2000)
    ap.add_argument("--max-steps", type=int, default=1_000_000)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    import torch
    from . import inputs
    from . import warmstart as W

    t0 = time.perf_counter()
    draws = inputs.warmstart_draws(args.train, seed=0)
    log("drew %d cavities (%.1f s)" % (len(draws), time.perf_counter() - t0))
    batch = W.Batch(draws)
    batch.start_from_rest()
    wall = batch.run(args.tol, check_every=args.check, max_steps=args.max_steps, chunk=20_000,
                     log=log, record_nu=False)
    n_lu = int(batch.steps.sum()) * 128 * 128
    log("steady states: %.1f s, %d node updates (%.0f MLUPS), steps median %d max %d, "
        "not steady %d, diverged %d" % (wall, n_lu, n_lu / wall / 1e6, np.median(batch.steps),
                                        batch.steps.max(),
                                        int((batch.status == 6).sum()),
                                        int((batch.status == 4).sum())))
    keep = batch.status != 4
    fields = batch.fields()[keep]
    batch.solver.close()
    del batch
    torch.cuda.empty_cache()
    eps = np.stack([d["eps"] for d in draws]).astype(np.float32)[keep]
    groups = np.stack([W.groups_of(d) for d in draws])[keep]
    sur = W.Surrogate(n=128, seed=0)
    t1 = time.perf_counter()
    losses = sur.train(eps, groups, fields, args.epochs, batch=args.batch, lr=args.lr, log=log)
    torch.cuda.synchronize()
    ttrain = time.perf_counter() - t1
    log("training: %.1f s, final loss %.3e" % (ttrain, losses[-1]))
    meta = dict(train=int(keep.sum()), epochs=args.epochs, batch=args.batch, lr=args.lr,
                tol=args.tol, losses=losses, datagen_s=wall, train_s=ttrain,
                samples_per_s=args.epochs * int(keep.sum()) / ttrain)
    if args.out:
        save_weights(args.out, sur.net, meta)
        log("saved", args.out)
    return meta


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
