"""Learned warm start: training on solves the method generates, and use as the
CG starting tensor (the warm-start form built on the convolution row of
Table 1 and the derivative rule of App. A.8).

Everything here drives the library through its C ABI: the samples' right-hand
sides come from the library's forward chain and RHS chain, the targets from
its CG solver, the network's forward, loss, backward and Adam step from its
kernels.  torch provides device memory and the random fields only.

Command line (one GPU):
    python -m paper_1001_5460_amd.warmstart train --samples 10000 --out ckpt.npz
    python -m paper_1001_5460_amd.warmstart eval --ckpt ckpt.npz --seeds 10000:10100
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import _lib as L

C, WIDTH = 32, 5


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the warm start runs on a HIP device")
    return torch


class Sampler:
    """Right-hand sides of one problem family: X_true a blob field, Y = the
    forward chain of X_true plus N(0, sigma^2) noise, B = the RHS chain of Y.
    The factors (and the operator handle) are shared by all samples."""

    def __init__(self, n, m, lam, sigma=0.01, blob_noise=0.1):
        import workload

        self.n, self.m = tuple(n), tuple(m)
        self.lam, self.sigma, self.blob_noise = lam, sigma, blob_noise
        A, D = workload.factors(self.n, self.m)
        self.op = L.Operator(A, D, lam)

    def rhs(self, seed):
        torch = _torch()
        import workload

        X, gen = workload.blob_field_torch(self.n, seed, self.blob_noise)
        Y = self.op.forward(X, chain="f32")
        Y += self.sigma * torch.randn(self.m, generator=gen, device=Y.device, dtype=torch.float32)
        return self.op.rhs(Y, chain="f32")

    def target(self, B, rtol=1e-5, max_iter=5000):
        """FP32 CG solution from zero (the training target)."""
        X, info = self.op.solve(B, precision="f32", rtol=rtol, max_iter=max_iter)
        return X, info


class WarmStart:
    """Owning wrapper of a cta_ws network handle."""

    def __init__(self, n, blocks=5, seed=0, params=None):
        self.n = tuple(int(v) for v in n)
        self.blocks = blocks
        self.handle = L.cta_ws_create(self.n, C, WIDTH, blocks, seed)
        if params is not None:
            L.cta_ws_params(self.handle, params, set=1)
        torch = _torch()
        self._dX0 = torch.empty(self.n, dtype=torch.float32, device="cuda")
        self._X0 = torch.empty(self.n, dtype=torch.float32, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")

    def close(self):
        if self.handle:
            L.cta_ws_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        return L.cta_ws_params(self.handle)

    def __call__(self, B, X0=None):
        """X0 = network(B) (F32 in, F32 out)."""
        if X0 is None:
            X0 = _torch().empty_like(B)
        return L.cta_ws_forward(self.handle, B, X0)

    def accumulate(self, B, T):
        """Forward, loss and backward of one sample (gradient accumulates);
        the loss is added to the device scalar self.loss."""
        L.cta_ws_forward(self.handle, B, self._X0, training=True)
        torch = _torch()
        li = torch.zeros(1, dtype=torch.float64, device="cuda")
        L.cta_ws_mse(self.handle, self._X0, T, self._dX0, li)
        L.cta_ws_backward(self.handle, self._dX0)
        self.loss += li

    def zero_grad(self):
        L.cta_ws_zero_grad(self.handle)

    def step(self, lr):
        L.cta_ws_adam_step(self.handle, lr, 0.9, 0.999, 1e-8)

    def save(self, path, meta):
        np.savez(path, params=self.params(), n=np.array(self.n), blocks=self.blocks,
                 meta=json.dumps(meta))

    @classmethod
    def load(cls, path):
        z = np.load(path, allow_pickle=False)
        return cls(tuple(int(v) for v in z["n"]), int(z["blocks"]), params=z["params"]), \
            json.loads(str(z["meta"]))


def lr_at(step, total, lr0, lr_min=1e-5, warmup=50):
    if step < warmup:
        return lr0 * (step + 1) / warmup
    t = (step - warmup) / max(1, total - warmup)
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * min(1.0, t)))


def validation_loss(net, smp, pairs):
    """Mean loss of the network over fixed (B, X*) pairs."""
    torch = _torch()
    tot = torch.zeros(1, dtype=torch.float64, device="cuda")
    li = torch.zeros(1, dtype=torch.float64, device="cuda")
    for B, T in pairs:
        L.cta_ws_forward(net.handle, B, net._X0)
        L.cta_ws_mse(net.handle, net._X0, T, net._dX0, li)
        tot += li
    return float(tot.item()) / max(1, len(pairs))


def train(n, m, lam, samples, batch=4, blocks=5, lr=1e-3, seed0=0, target_rtol=1e-5,
          log_every=100, log=print, net_seed=0, smp=None, net=None):
    """Train a network (fresh unless given) on `samples` generated solves
    (seeds seed0..); every sample is used once.  The logged loss is the mean
    over the samples since the previous log line.  Returns the network, the
    sampler and a training record."""
    torch = _torch()
    smp = smp or Sampler(n, m, lam)
    net = net or WarmStart(n, blocks, net_seed)
    steps = samples // batch
    hist, t0 = [], time.time()
    solve_s = train_s = 0.0
    iters = []
    net.loss.zero_()
    since = 0
    for st in range(steps):
        net.zero_grad()
        for j in range(batch):
            seed = seed0 + st * batch + j
            ta = time.time()
            B = smp.rhs(seed)
            T, info = smp.target(B, target_rtol)
            torch.cuda.synchronize()
            tb = time.time()
            iters.append(info["iters"])
            net.accumulate(B, T)
            torch.cuda.synchronize()
            solve_s += tb - ta
            train_s += time.time() - tb
        net.step(lr_at(st, steps, lr))
        since += batch
        if (st + 1) % log_every == 0 or st == steps - 1:
            loss = float(net.loss.item()) / since
            net.loss.zero_()
            since = 0
            hist.append((st, loss))
            log(f"step {st}/{steps} samples {(st + 1) * batch} loss {loss:.4e} "
                f"target iters {np.mean(iters[-batch:]):.0f} elapsed {time.time() - t0:.0f}s")
    torch.cuda.synchronize()
    rec = {"samples": steps * batch, "batch": batch, "blocks": blocks, "lr": lr,
           "target_rtol": target_rtol, "seeds": [seed0, seed0 + steps * batch - 1],
           "loss_history": hist, "seconds": time.time() - t0,
           "data_seconds": solve_s, "train_seconds": train_s,
           "mean_target_iters": float(np.mean(iters)), "n": list(n), "m": list(m), "lam": lam}
    return net, smp, rec


def evaluate(net, smp, seeds, rtol=1e-8, precision="bf16_reliable", inner_rtol=0.1, log=print,
             keep=0):
    """Solve each held-out seed's problem from zero and from the network's
    start (fallback to zero if the start is worse), to `rtol`; report
    iterations and wall time (network inference included for the warm start).
    With keep > 0 also return (B, X_zero, X_warm) of the first `keep` seeds."""
    torch = _torch()
    rows, kept = [], []
    for seed in seeds:
        B32 = smp.rhs(seed)
        B = B32.double()
        torch.cuda.synchronize()
        # zero start
        Xz = torch.zeros_like(B)
        t0 = time.perf_counter()
        _, iz = smp.op.solve(B, Xz, precision=precision, rtol=rtol, max_iter=20000,
                             inner_rtol=inner_rtol, max_refine=200)
        tz = time.perf_counter() - t0
        # warm start: network inference + solve
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X0 = net(B32)
        Xw = X0.double()
        _, iw = smp.op.solve(B, Xw, precision=precision, rtol=rtol, max_iter=20000, x0_given=1,
                             fallback_zero=1, inner_rtol=inner_rtol, max_refine=200)
        tw = time.perf_counter() - t0
        # relative residual of the network's start alone
        r0 = _rel_res(smp.op, B, X0.double())
        rows.append({"seed": seed, "zero_iters": iz["iters"], "warm_iters": iw["iters"],
                     "zero_s": tz, "warm_s": tw, "zero_res": iz["rel_res_true"],
                     "warm_res": iw["rel_res_true"], "start_res": r0,
                     "zero_status": iz["status"], "warm_status": iw["status"]})
        log(f"seed {seed}: iters zero {iz['iters']} warm {iw['iters']}  time zero {tz * 1e3:.1f} ms "
            f"warm {tw * 1e3:.1f} ms  start residual {r0:.3e}")
        if len(kept) < keep:
            kept.append((B, Xz, Xw))
    return (rows, kept) if keep else rows


def _rel_res(op, B, X):
    Q = op.apply(X, chain="f64")
    return float((B - Q).norm() / B.norm())


def summarize(rows):
    zi = np.array([r["zero_iters"] for r in rows], dtype=float)
    wi = np.array([r["warm_iters"] for r in rows], dtype=float)
    zt = np.array([r["zero_s"] for r in rows])
    wt = np.array([r["warm_s"] for r in rows])
    return {"problems": len(rows), "zero_iters_mean": zi.mean(), "warm_iters_mean": wi.mean(),
            "iters_saved_frac": 1.0 - wi.sum() / zi.sum(), "zero_s_mean": zt.mean(),
            "warm_s_mean": wt.mean(), "time_speedup": zt.sum() / wt.sum(),
            "start_res_median": float(np.median([r["start_res"] for r in rows])),
            "all_converged": all(r["zero_status"] == 0 and r["warm_status"] == 0 for r in rows)}


def _seeds(spec):
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


def main(argv=None):
    import workload

    cfg = workload.CONFIGS[4]
    ap = argparse.ArgumentParser(prog="python -m paper_1001_5460_amd.warmstart")
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--samples", type=int, default=10000)
    tr.add_argument("--batch", type=int, default=4)
    tr.add_argument("--blocks", type=int, default=5)
    tr.add_argument("--lr", type=float, default=1e-3)
    tr.add_argument("--log-every", type=int, default=100)
    tr.add_argument("--out", required=True)
    tr.add_argument("--eval-seeds", default="10000:10100")
    ev = sub.add_parser("eval")
    ev.add_argument("--ckpt", required=True)
    ev.add_argument("--seeds", default="10000:10100")
    for p in (tr, ev):
        p.add_argument("--json", default=None, help="write the evaluation summary here")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    n, m, lam = cfg["n"], cfg["m"], cfg["lam"]
    if a.cmd == "train":
        net, smp, rec = train(n, m, lam, a.samples, a.batch, a.blocks, a.lr, log=log,
                              log_every=a.log_every)
        net.save(a.out, rec)
        log(f"saved {a.out}")
        seeds = _seeds(a.eval_seeds)
    else:
        net, rec = WarmStart.load(a.ckpt)
        smp = Sampler(n, m, lam)
        seeds = _seeds(a.seeds)
    rows = evaluate(net, smp, seeds, cfg["rtol"], log=log)
    summ = summarize(rows)
    log(json.dumps(summ))
    if a.json:
        with open(a.json, "w") as f:
            json.dump({"summary": summ, "rows": rows, "training": rec}, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
