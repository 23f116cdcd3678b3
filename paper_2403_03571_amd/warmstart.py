"""Training and evaluation driver of the learned warm start (2D).

    python -m paper_2403_03571_amd.warmstart --train 20000 --test 1000 \
        --out warmstart_params.npz

1. Training data: instances of the warm-start workload (512x512 pixels,
   N ~ U{200..1000}, det-1 anisotropy with aspect U[1,3], equal volumes) are
   fitted to 1 % from W_0 = 0 by the batched solver; their per-seed features
   and targets t = N (w* - mean w*) are formed on the device by the library.
2. Training: Adam on minibatches of seeds (the library's forward, backward
   and update kernels).
3. Evaluation on held-out instances: the plain cold-start fit (W_0 = 0, as
   Algorithm 2 of arXiv 2403.03571) against the warm-start fit (predicted
   W_0, cold start as fallback), both through the library and both
   certified by their own stopping rule: passes, iterations and seconds to
   1 %, per instance and summarised.

Only the arithmetic of the method runs in the library's kernels; torch is
used to hold device arrays, concatenate them and draw minibatches.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TRAIN_SEED0 = 500000
TEST_SEED0 = 600000


def init_params(seed: int) -> np.ndarray:
    """He-uniform initial weights, zero biases, layer by layer (W [in][out]
    row-major, then b) for 20 -> 128 -> 128 -> 128 -> 1."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in ((20, 128), (128, 128), (128, 128), (128, 1)):
        lim = np.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, i * o))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def make_data(ctx, net, seeds, batch=256, log=print):
    """Fit the instances with the batched solver; return device tensors of
    features (S, 20) and targets (S,)."""
    import torch

    import apd_synth as S
    import paper_2403_03571_amd as apd
    feats, targs = [], []
    t0 = time.perf_counter()
    nfit = 0
    for k in range(0, len(seeds), batch):
        insts = [S.make_c5(s) for s in seeds[k:k + batch]]
        probs = [apd.Problem.from_instance(i, "cuda:0") for i in insts]
        ws, reps, status = ctx.apd_fit_weights_batched(probs)
        for p, w, r in zip(probs, ws, reps):
            if not r.converged:
                continue
            feats.append(net.features(p))
            targs.append(net.targets(w))
            nfit += 1
        log(f"# data: {min(k + batch, len(seeds))}/{len(seeds)} instances fitted "
            f"({time.perf_counter() - t0:.1f} s)")
    return torch.cat(feats), torch.cat(targs), nfit, time.perf_counter() - t0


def train(net, F, t, epochs=20, batch=4096, lr=1e-3, seed=0, log=print):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = F.shape[0]
    hist = []
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(F.device)
        # cosine decay from lr to lr / 20
        lr_ep = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * ep / max(1, epochs))))
        tot, cnt = 0.0, 0
        for k in range(0, n - batch + 1, batch):
            idx = perm[k:k + batch]
            Fb = F.index_select(0, idx).contiguous()
            tb = t.index_select(0, idx).contiguous()
            tot += net.train_step(Fb, tb, lr_ep)
            cnt += 1
            step += 1
        hist.append(tot / max(cnt, 1))
        log(f"# epoch {ep}: mean minibatch loss {hist[-1]:.4g} (lr {lr_ep:.2g}, "
            f"{time.perf_counter() - t0:.1f} s)")
    return hist, time.perf_counter() - t0


def evaluate(ctx, net, seeds, log=print):
    """Cold vs warm fit on each held-out instance."""
    import torch

    import apd_synth as S
    import paper_2403_03571_amd as apd
    rows = []
    for s in seeds:
        inst = S.make_c5(s)
        p = apd.Problem.from_instance(inst, "cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wc, rc = ctx.apd_fit_weights(p)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        t0 = time.perf_counter()
        ww, rw, used = net.fit(p)
        torch.cuda.synchronize()
        tw = time.perf_counter() - t0
        rows.append({"seed": s, "n": inst.n, "cold_evals": rc.evals, "cold_iters": rc.iters,
                     "cold_s": tc, "cold_ok": rc.converged, "warm_evals": rw.evals,
                     "warm_iters": rw.iters, "warm_s": tw, "warm_ok": rw.converged,
                     "warm_used": used})
    ce = np.array([r["cold_evals"] for r in rows], float)
    we = np.array([r["warm_evals"] for r in rows], float)
    ct = np.array([r["cold_s"] for r in rows])
    wt = np.array([r["warm_s"] for r in rows])
    ratio = we / ce
    summ = {
        "instances": len(rows),
        "cold_converged": int(sum(r["cold_ok"] for r in rows)),
        "warm_converged": int(sum(r["warm_ok"] for r in rows)),
        "warm_kept": int(sum(r["warm_used"] for r in rows)),
        "cold_evals_mean": float(ce.mean()), "warm_evals_mean": float(we.mean()),
        "evals_ratio_median": float(np.median(ratio)),
        "evals_ratio_p10_p90": [float(np.percentile(ratio, 10)), float(np.percentile(ratio, 90))],
        "cold_seconds_total": float(ct.sum()), "warm_seconds_total": float(wt.sum()),
        "warm_faster_fraction": float(np.mean(wt < ct)),
    }
    log(f"# eval: {json.dumps(summ)}")
    return summ, rows


def batched_compare(ctx, net, seeds, log=print):
    """The same held-out instances in one batched solve, cold vs warm."""
    import torch

    import apd_synth as S
    import paper_2403_03571_amd as apd
    probs = [apd.Problem.from_instance(S.make_c5(s), "cuda:0") for s in seeds]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rc, stc = ctx.apd_fit_weights_batched(probs)
    torch.cuda.synchronize()
    tc = time.perf_counter() - t0
    t0 = time.perf_counter()
    ws = [net.predict(p) for p in probs]
    _, rw, stw = ctx.apd_fit_weights_batched(probs, ws=ws)
    torch.cuda.synchronize()
    tw = time.perf_counter() - t0
    out = {"instances": len(probs), "cold_seconds": tc, "warm_seconds": tw,
           "cold_status": stc, "warm_status": stw,
           "cold_max_evals": max(r.evals for r in rc), "warm_max_evals": max(r.evals for r in rw),
           "cold_evals_mean": float(np.mean([r.evals for r in rc])),
           "warm_evals_mean": float(np.mean([r.evals for r in rw]))}
    log(f"# batched: {json.dumps(out)}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--test", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default="warmstart_params.npz")
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    import torch

    import paper_2403_03571_amd as apd
    torch.cuda.set_device(0)
    ctx = apd.Context(0)
    net = apd.WarmStart(ctx, init_params(0))
    log = lambda m: print(m, file=sys.stderr, flush=True)
    F, t, nfit, data_s = make_data(ctx, net, list(range(TRAIN_SEED0, TRAIN_SEED0 + args.train)), log=log)
    hist, train_s = train(net, F, t, epochs=args.epochs, lr=args.lr, log=log)
    np.savez(args.out, params=net.params(), meta=json.dumps({
        "train_instances": nfit, "samples": int(F.shape[0]), "epochs": args.epochs,
        "loss_history": hist}))
    test = list(range(TEST_SEED0, TEST_SEED0 + args.test))
    summ, rows = evaluate(ctx, net, test, log=log)
    bat = batched_compare(ctx, net, test[:min(len(test), 512)], log=log)
    rep = {"train_instances": nfit, "samples": int(F.shape[0]), "data_seconds": data_s,
           "train_seconds": train_s, "loss_first_last": [hist[0], hist[-1]], "eval": summ,
           "batched": bat}
    print(json.dumps(rep), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"summary": rep, "rows": rows}, f)


if __name__ == "__main__":
    main()
