"""Learned initial guess: training data produced by the solver, training on the GPU, evaluation.

The network and every kernel it runs are in csrc/net.hip (entry points dda_net_* and dda_guess);
this module only orchestrates them:

  * build_dataset: random particles (inputs.c5_particle), each solved by plain QMR from a zero
    guess; the network's features and the target (exciting field minus incident field at the
    dipoles) are written on the device by the library.
  * train: Adam on shuffled mini-batches, cosine-decayed learning rate.
  * evaluate: for held-out particles, QMR iterations and wall time to the tolerance from a zero
    guess and from the network's guess (time includes building the features and the forward
    pass; a guess that does not lower the residual below |b| is replaced by zero inside the
    solver, dda_solve_opts.x0_check).

    python -m paper_0704_0037_amd.learned_guess --grid 48 --train 2000 --eval 200
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import dda, inputs

# (input channels, output channels) of the eight convolutions, in the parameter layout order
LAYERS = ((16, 16), (16, 32), (32, 48), (48, 64), (64, 48), (48, 32), (32, 16), (16, 6))


def init_params(seed, head_scale=0.0):
    """He-normal weights (std sqrt(2 / (27 cin))), zero biases; the head is scaled by head_scale
    (0 by default: the untrained network outputs zero, i.e. the guess x0 = b)."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ci, co) in enumerate(LAYERS):
        w = rng.standard_normal(27 * co * ci) * np.sqrt(2.0 / (27 * ci))
        if li == len(LAYERS) - 1:
            w *= head_scale
        parts += [w, np.zeros(co)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == dda.num_params()
    return p


def _log(msg, quiet):
    if not quiet:
        print(f"learned_guess: {msg}", file=sys.stderr, flush=True)


def build_dataset(net, seeds, tol=1e-5, quiet=True):
    """Features [n][G^3][16] (bf16) and targets [n][G^3][6] (f32) of the particles `seeds`."""
    n, cells = len(seeds), net.cells
    feats = torch.empty((n, cells, 16), dtype=torch.bfloat16, device=net.device)
    tgts = torch.empty((n, cells, 6), dtype=torch.float32, device=net.device)
    iters = []
    t0 = time.perf_counter()
    for i, s in enumerate(seeds):
        mask, m, kd, beam = inputs.c5_particle(s, net.grid)
        with dda.Context(mask, m, kd) as ctx:
            x, info, st = ctx.solve([beam], tol=tol, raise_on_fail=False)
            iters.append(info[0]["iters"])
            net.features(ctx, beam, feats[i])
            net.target(ctx, beam, x[0].contiguous(), tgts[i])
        if (i + 1) % 100 == 0:
            _log(f"solved {i + 1}/{n} particles ({time.perf_counter() - t0:.1f} s)", quiet)
    torch.cuda.synchronize()
    return feats, tgts, {"solve_s": time.perf_counter() - t0, "mean_iters": float(np.mean(iters))}


def train(net, feats, tgts, epochs, batch=8, lr=1e-3, seed=0, quiet=True):
    """Adam over shuffled mini-batches with a cosine-decayed learning rate; returns loss history."""
    n = feats.shape[0]
    rng = np.random.default_rng(seed)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    hist = []
    step = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(n)
        losses = []
        for k in range(steps_per_epoch):
            idx = torch.from_numpy(order[k * batch:(k + 1) * batch]).to(feats.device)
            f = feats.index_select(0, idx).contiguous()
            t = tgts.index_select(0, idx).contiguous()
            cur = lr * 0.5 * (1.0 + np.cos(np.pi * step / total))
            losses.append(net.train_step(f, t, max(cur, 1e-3 * lr)))
            step += 1
        hist.append(float(np.mean(losses)))
        if (ep + 1) % max(1, epochs // 10) == 0:
            _log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.4g} ({time.perf_counter() - t0:.1f} s)", quiet)
    return hist


def evaluate(net, seeds, tol=1e-5, quiet=True):
    """Zero guess vs learned guess on held-out particles."""
    rows = []
    for i, s in enumerate(seeds):
        mask, m, kd, beam = inputs.c5_particle(s, net.grid)
        with dda.Context(mask, m, kd) as ctx:
            # warm the context's buffers so both timings see the same state
            ctx.solve([beam], tol=1e-1, raise_on_fail=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x0z, iz, sz = ctx.solve([beam], tol=tol, raise_on_fail=False)
            torch.cuda.synchronize()
            tz = time.perf_counter() - t0
            t0 = time.perf_counter()
            g = net.guess(ctx, [beam])
            xg, ig, sg = ctx.solve([beam], tol=tol, x0=g, x0_check=True, raise_on_fail=False)
            torch.cuda.synchronize()
            tg = time.perf_counter() - t0
            b = ctx.rhs(beam)
            nb = torch.linalg.norm(b)
            r0 = float(torch.linalg.norm(b - ctx.matvec(beam, g[0].contiguous())) / nb)
            # the untrained network's guess, x0 = b (zero output), as a second baseline
            rb = float(torch.linalg.norm(b - ctx.matvec(beam, b)) / nb)
            xb, ib, sb = ctx.solve([beam], tol=tol, x0=b.reshape(1, 3, ctx.n), x0_check=True, raise_on_fail=False)
        rows.append({"seed": int(s), "n": int(ctx.n), "m": m.real, "kd": kd, "iters_zero": iz[0]["iters"],
                     "iters_guess": ig[0]["iters"], "iters_b": ib[0]["iters"], "t_zero_s": tz, "t_guess_s": tg,
                     "res0_guess": r0, "res0_b": rb, "fallback": bool(not r0 < 1.0), "status": [sz, sg, sb]})
        if (i + 1) % 50 == 0:
            _log(f"evaluated {i + 1}/{len(seeds)}", quiet)
    iz = np.array([r["iters_zero"] for r in rows], dtype=np.float64)
    ig = np.array([r["iters_guess"] for r in rows], dtype=np.float64)
    tz = np.array([r["t_zero_s"] for r in rows])
    tg = np.array([r["t_guess_s"] for r in rows])
    return {
        "particles": len(rows),
        "mean_iters_zero": float(iz.mean()), "mean_iters_guess": float(ig.mean()),
        "iteration_ratio": float(ig.sum() / iz.sum()),
        "median_iteration_ratio": float(np.median(ig / np.maximum(iz, 1))),
        "time_zero_s": float(tz.sum()), "time_guess_s": float(tg.sum()), "speedup": float(tz.sum() / tg.sum()),
        "fewer_iterations_fraction": float(np.mean(ig < iz)),
        "fallbacks": int(sum(r["fallback"] for r in rows)),
        "mean_res0_guess": float(np.mean([r["res0_guess"] for r in rows])),
        "mean_res0_b": float(np.mean([r["res0_b"] for r in rows])),
        "mean_iters_b": float(np.mean([r["iters_b"] for r in rows])),
        "rows": rows,
    }


def run(grid=48, n_train=2000, n_eval=200, epochs=20, batch=8, lr=1e-3, seed=5000, tol=1e-5, quiet=False):
    params = init_params(seed)
    with dda.Net(grid, params, max_batch=batch) as net:
        _log(f"building {n_train} training particles on a {grid}^3 box", quiet)
        feats, tgts, dstat = build_dataset(net, range(seed, seed + n_train), tol, quiet)
        t0 = time.perf_counter()
        hist = train(net, feats, tgts, epochs, batch, lr, seed, quiet)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        del feats, tgts
        _log(f"evaluating on {n_eval} held-out particles", quiet)
        ev = evaluate(net, range(seed + 10 ** 6, seed + 10 ** 6 + n_eval), tol, quiet)
        ev.update({"grid": grid, "train_particles": n_train, "epochs": epochs, "batch": batch, "lr": lr,
                   "train_s": t_train, "dataset": dstat, "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]})
        return ev, net.params()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=48)
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--eval", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=5000)
    ap.add_argument("--rows", action="store_true", help="print the per-particle rows too")
    ap.add_argument("--save-params", default="", help="write the trained parameters (float32 .npy)")
    a = ap.parse_args()
    ev, p = run(a.grid, a.train, a.eval, a.epochs, a.batch, a.lr, a.seed)
    if a.save_params:
        np.save(a.save_params, p)
    if not a.rows:
        ev.pop("rows")
    print(json.dumps(ev), flush=True)


if __name__ == "__main__":
    main()
