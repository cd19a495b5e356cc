"""Learned warm start of the porous-cavity solver.

A convolutional encoder-decoder (nn.UNet) is trained on steady states that
the solver itself produces for cavities with random porosity maps and
dimensionless groups; its prediction initialises new cavities
(clb_set_state_device: f = f^eq(1, u), g = g^eq(T, u)), which then run to the
same steady state in fewer steps.  The paper starts from rest; this is an
addition for many-query use.

Everything numerical runs in the HIP library (solver, network, loss,
optimizer); this module drives it: it builds the parameter sets, moves data
between host and device, and schedules the runs.
"""
import ctypes as C
import math
import time

import numpy as np

from . import _binding as B
from . import inputs, nn, workloads

MA = 0.1
U_C = MA / math.sqrt(3.0)  # velocity scale of the cavity scaling: Ma c_s (Eq. 46)
NGROUPS = 4


def groups_of(d):
    """Normalised dimensionless groups of one draw (network input channels)."""
    return np.array([(math.log10(d["Ra"]) - 5.0) / 2.0, (math.log10(d["Da"]) + 3.0) / 2.0,
                     (math.log10(d["Pr"]) - 0.35) / 0.5, (d["sigma"] - 1.0) / 0.2],
                    dtype=np.float32)


def case_of(d, storage="f32"):
    """Cavity parameters of one draw: hot west wall, cold east wall,
    adiabatic top and bottom, porosity map with Kozeny-Carman K and Ergun
    F_phi per node for the drawn mean Darcy number."""
    n = d["n"]
    dp = inputs.particle_diameter_for_mean_Da(d["eps"], d["Da"], n - 1)
    return workloads.cavity(n, Ra=d["Ra"], Pr=d["Pr"], sigma=d["sigma"], Da=d["Da"],
                            eps=d["eps"], dp=dp, storage=storage, Ma=MA)


class Batch:
    """Many cavities in one solver context, run to steady state in chunks
    (clb_run) with progress reports between chunks."""

    def __init__(self, draws, storage="f32", launch=(128, 2, 0), stream=None):
        self.draws = draws
        self.cases = [case_of(d, storage) for d in draws]
        self.solver = B.Solver(self.cases, stream=stream)
        if launch:
            self.solver.set_launch(*launch)
        self.count = len(draws)
        self.steps = np.zeros(self.count, dtype=np.int64)
        self.status = np.full(self.count, B.NOT_CONVERGED, dtype=np.int32)
        self.nu = [[] for _ in range(self.count)]

    def start_from_rest(self):
        for k, d in enumerate(self.draws):
            self.solver.set_state(k, inputs.cavity_initial_T(d["n"], seed=1))

    def run(self, tol, check_every=1000, max_steps=2_000_000, chunk=100_000, log=None,
            record_nu=True):
        s = self.solver
        t0 = time.perf_counter()
        done = 0
        while done < max_steps and np.any(self.status == B.NOT_CONVERGED):
            m = min(chunk, max_steps - done)
            rounds = (m + check_every - 1) // check_every
            r = s.run(m, check_every=check_every, tol=tol,
                      nu_side=B.WEST if record_nu else None,
                      max_records=rounds if record_nu else 0)
            live = self.status == B.NOT_CONVERGED
            self.steps[live] += r["steps"][live]
            fin = live & (r["status"] != B.NOT_CONVERGED)
            self.status[fin] = r["status"][fin]
            if record_nu:
                for k in np.nonzero(live)[0]:
                    rec = r["nu"][k]
                    self.nu[k].extend(rec[np.isfinite(rec)].tolist())
            done += m
            if log:
                log("  %d steps, %d of %d steady, %d diverged, %.1f s"
                    % (done, int((self.status == B.OK).sum()), self.count,
                       int((self.status == B.ERR_DIVERGED).sum()), time.perf_counter() - t0))
        s.synchronize()
        return time.perf_counter() - t0

    def fields(self):
        """(count, n*n, 3) FP32: u / u_c, v / u_c, T - 1/2 of every domain."""
        out = []
        for k in range(self.count):
            m = self.solver.macros(k)
            out.append(np.stack([m["ux"] / U_C, m["uy"] / U_C, m["T"] - 0.5], axis=-1)
                       .reshape(-1, 3).astype(np.float32))
        return np.stack(out)


class Surrogate:
    """The network plus its device-resident training data."""

    def __init__(self, n=128, seed=0, stream=None):
        import torch
        self.torch = torch
        self.n = n
        self.net = nn.UNet(levels=5, base=16, cin=16, cout=16, seed=seed, stream=stream)

    def _features(self, eps_d, groups_d, idx_d, batch):
        x = self.torch.empty(batch * self.n * self.n * 16, dtype=self.torch.bfloat16,
                             device=self.net.device)
        nn.call("clb_nn_features", nn.ptr(eps_d), nn.ptr(groups_d), NGROUPS, nn.ptr(idx_d),
                batch, self.n, self.n, nn.ptr(x), C.c_void_p(self.net.stream.cuda_stream))
        return x

    def train(self, eps, groups, fields, epochs, batch=32, lr=2e-3, wd=1e-4, seed=0, log=None):
        """eps (S, n, n), groups (S, NGROUPS), fields (S, n*n, 3), FP32 host
        arrays.  AdamW with a cosine learning-rate decay.  Returns the mean
        loss of every epoch."""
        torch = self.torch
        dev = self.net.device
        S = eps.shape[0]
        eps_d = torch.tensor(eps, dtype=torch.float32, device=dev)
        groups_d = torch.tensor(groups, dtype=torch.float32, device=dev)
        fields_d = torch.tensor(fields, dtype=torch.float32, device=dev)
        tgt = torch.empty(batch * self.n * self.n * 3, dtype=torch.float32, device=dev)
        r = np.random.Generator(np.random.PCG64(seed))
        nb = S // batch
        total = epochs * nb
        losses = []
        stream = C.c_void_p(self.net.stream.cuda_stream)
        acc = torch.zeros(1, dtype=torch.float64, device=dev)
        it = 0
        t0 = time.perf_counter()
        for ep in range(epochs):
            perm = r.permutation(S).astype(np.int32)
            idx_all = torch.tensor(perm, device=dev)
            acc.zero_()
            for b in range(nb):
                idx = idx_all[b * batch:(b + 1) * batch]
                x = self._features(eps_d, groups_d, idx, batch)
                nn.call("clb_nn_gather", nn.ptr(fields_d), 3, nn.ptr(idx), batch,
                        self.n * self.n, nn.ptr(tgt), stream)
                self.net.forward(x, batch, self.n, self.n)
                loss = self.net.backward(tgt, 3, batch, self.n, self.n)
                acc += loss
                step_lr = 0.5 * lr * (1.0 + math.cos(math.pi * it / total))
                self.net.adamw(step_lr, wd=wd)
                it += 1
            losses.append(acc.item() / nb)
            if log:
                log("  epoch %d loss %.3e (%.1f s)" % (ep, losses[-1], time.perf_counter() - t0))
        return losses

    def predict(self, eps, groups):
        """Network output for the given maps and groups: FP32 device tensor
        (S, n, n, 16); channels 0..2 are u / u_c, v / u_c, T - 1/2."""
        torch = self.torch
        dev = self.net.device
        S = eps.shape[0]
        eps_d = torch.tensor(eps, dtype=torch.float32, device=dev)
        groups_d = torch.tensor(groups, dtype=torch.float32, device=dev)
        idx = torch.arange(S, dtype=torch.int32, device=dev)
        x = self._features(eps_d, groups_d, idx, S)
        out = self.net.forward(x, S, self.n, self.n)
        return out.clone()

    def warm_start(self, batch, out):
        """Initialise every domain of a Batch from the prediction `out`; the
        solver stream waits for the network's work first."""
        self.net.stream.synchronize()
        per = self.n * self.n * 16
        for k in range(batch.count):
            nn.call("clb_set_state_device", batch.solver._ctx, k,
                    C.c_void_p(out.data_ptr() + 4 * per * k), 16, U_C, 0.5)
        batch.solver.synchronize()


def settle_steps(nu, nu_inf, every, tol=1e-4):
    """Steps after which the recorded Nusselt numbers stay within tol of
    nu_inf (records every `every` steps); None if the last record is not."""
    nu = np.asarray(nu)
    if nu.size == 0 or abs(nu[-1] - nu_inf) > tol:
        return None
    off = np.nonzero(np.abs(nu - nu_inf) > tol)[0]
    # record i is taken after (i + 1) * every steps
    return int((off[-1] + 2) * every) if off.size else every


def evaluate(sur, draws, tol=1e-9, check_every=5000, max_steps=3_000_000, log=None):
    """Held-out comparison of starting from rest and from the network's
    prediction.  Both runs go to the same residual tolerance; the reference
    steady Nusselt number Nu_inf of each cavity is the final value of the run
    from rest.  Time to steady state = steps after which the hot-wall Nusselt
    number stays within 1e-4 of Nu_inf.  A warm run that diverges is restarted
    from rest (res["fallback"] counts them)."""
    eps = np.stack([d["eps"] for d in draws]).astype(np.float32)
    groups = np.stack([groups_of(d) for d in draws])
    res = {}
    plain = Batch(draws)
    plain.start_from_rest()
    if log:
        log("from rest:")
    res["wall_plain"] = plain.run(tol, check_every, max_steps, log=log)
    nu_inf = np.array([x[-1] if x else np.nan for x in plain.nu])
    f_plain = plain.fields()
    warm = Batch(draws)
    t0 = time.perf_counter()
    out = sur.predict(eps, groups)
    sur.warm_start(warm, out)
    res["inference_s"] = time.perf_counter() - t0
    pred = out.cpu().numpy().reshape(len(draws), -1, 16)[..., :3]
    if log:
        log("from the prediction (inference %.3f s):" % res["inference_s"])
    res["wall_warm"] = warm.run(tol, check_every, max_steps, log=log)
    sw = [settle_steps(warm.nu[k], nu_inf[k], check_every) for k in range(len(draws))]
    # A warm start that diverges falls back to a run from rest; its time to
    # steady state counts the steps lost before the divergence.
    fb = [k for k in range(len(draws)) if warm.status[k] == B.ERR_DIVERGED]
    res["fallback"] = len(fb)
    if fb:
        if log:
            log("fallback to rest for %d cavities" % len(fb))
        redo = Batch([draws[k] for k in fb])
        redo.start_from_rest()
        res["wall_warm"] += redo.run(tol, check_every, max_steps, log=log)
        for j, k in enumerate(fb):
            st = settle_steps(redo.nu[j], nu_inf[k], check_every)
            sw[k] = None if st is None else int(warm.steps[k]) + st
            warm.steps[k] += redo.steps[j]
            warm.status[k] = redo.status[j]
            warm.nu[k] = redo.nu[j]
        redo.solver.close()
    nu_w = np.array([x[-1] if x else np.nan for x in warm.nu])
    sp = [settle_steps(plain.nu[k], nu_inf[k], check_every) for k in range(len(draws))]
    err = np.sqrt(((pred - f_plain) ** 2).sum(axis=(1, 2)) / (f_plain ** 2).sum(axis=(1, 2)))
    res.update(steps_plain=plain.steps.tolist(), steps_warm=warm.steps.tolist(),
               status_plain=plain.status.tolist(), status_warm=warm.status.tolist(),
               settle_plain=sp, settle_warm=sw, nu_plain=nu_inf.tolist(), nu_warm=nu_w.tolist(),
               pred_rel_l2=err.tolist())
    plain.solver.close()
    warm.solver.close()
    return res
