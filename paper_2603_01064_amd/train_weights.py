"""Offline training of per-level smoother weights on the GPU (Algorithm 5).

Each weight set belongs to one operator (grid, kernel width, alpha): the
paper trains smoothers for a fixed coefficient matrix and retrains when it
changes.  Training uses the library's own ``train_step`` (level-wise loss or
the combined cycle loss, hand-written adjoint, Adam) on batches of i.i.d. N(0,1) error vectors, an
optional rollout of k in 1..K cycles of the current smoothers before each
batch (Algorithm 5, DataGeneration) and a curriculum over alpha (weights of
a larger alpha initialise the next smaller one, Sec. 4.1).

Usage: python -m paper_2603_01064_amd.train_weights --n 255 --s 0.01 --levels 5 \
           --alphas 1e-2 1e-3 1e-4 --steps 1500 --out paper_2603_01064_amd/weights/grid255_s0.01.npz
       python -m paper_2603_01064_amd.train_weights levels --weights F.npz --set 1   (coarsest-level sweep)
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import inputs
from . import nmg

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def save_weights(path: str, meta: dict, sets: list) -> None:
    """``sets[k][l]`` is the flat FP32 weight vector of level l of set k."""
    arrs = {f"set{k}_level{l}": np.asarray(w, dtype=np.float32) for k, s in enumerate(sets) for l, w in enumerate(s)}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8), **arrs)


def load_weights(path: str):
    """Returns ``(meta, sets)`` written by :func:`save_weights`."""
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(bytes(z["meta"]).decode())
        sets = []
        k = 0
        while f"set{k}_level0" in z:
            lv = []
            l = 0
            while f"set{k}_level{l}" in z:
                lv.append(np.array(z[f"set{k}_level{l}"]))
                l += 1
            sets.append(lv)
            k += 1
    return meta, sets


def select_set(set_alphas, alpha: float) -> int:
    """Weight set for a request with regularisation `alpha`: the smallest
    trained alpha that is at least alpha / 2 (the largest set if none is).
    Measured at 255^2, s = 2.5h: a set trained at alpha_k keeps converging
    for requests down to alpha_k / 10 (more slowly) but diverges for
    requests more than about twice alpha_k."""
    ok = [i for i, a in enumerate(set_alphas) if a >= alpha / 2]
    if not ok:
        return max(range(len(set_alphas)), key=lambda i: set_alphas[i])
    return min(ok, key=lambda i: set_alphas[i])


def rollout(h: nmg.Handle, e: torch.Tensor, alpha: torch.Tensor, K: int, gen: torch.Generator,
            precision: str, use_fprime: bool = False, rescale: bool = False) -> torch.Tensor:
    """DataGeneration of Algorithm 5 on the device (``nmg_rollout``): each
    sample draws k ~ U{1..K} and goes through k cycles e <- e - NMG(0, A e)
    of the current smoothers (V(1, 0), F' as in training), without
    gradients.  ``rescale`` (off by default, not part of Algorithm 5) brings
    every sample back to unit RMS afterwards, so rolled-out samples weigh as
    much in the loss as fresh ones (the loss is homogeneous of degree two)."""
    if K <= 0:
        return e
    B = e.shape[0]
    ks = torch.randint(1, K + 1, (B,), generator=gen)
    h.rollout(e, alpha, ks.numpy(), nu1=1, nu2=0, use_fprime=use_fprime, precision=precision)
    if not rescale:
        return e
    rms = e.reshape(B, -1).norm(dim=1) / (e[0].numel() ** 0.5)
    return e / rms.clamp_min(1e-30).reshape(B, 1, 1)


def train_set(h: nmg.Handle, alpha_value: float, steps: int, batch: int, lr: float, mask: str, seed: int,
              rollout_K: int = 0, log_every: int = 100, precision: str = "fp32", use_fprime: bool = False,
              rollout_rescale: bool = False):
    dev = torch.device("cuda:0")
    n = h.problem.n
    alpha = torch.full((batch,), alpha_value, dtype=torch.float64, device=dev)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.time()
    for step in range(steps):
        e = torch.randn((batch, n, n), generator=gen, dtype=torch.float32).to(dev)
        e = rollout(h, e, alpha, rollout_K, gen, "mixed" if precision == "mixed" else "fp32", use_fprime,
                    rollout_rescale)
        cur_lr = lr * (0.1 ** (step / max(1, steps)))  # decays by 10x over the run
        losses = h.train_step(e, alpha, mask=mask, use_fprime=use_fprime, precision=precision, lr=cur_lr)
        hist.append(losses.tolist())
        if log_every and step % log_every == 0:
            print(f"  alpha={alpha_value:g} step {step} losses {np.array2string(losses, precision=3)} "
                  f"({time.time() - t0:.1f}s)", flush=True)
    return hist


def evaluate(h: nmg.Handle, alpha_value: float, batch: int, nu1: int, nu2: int, use_fprime: bool,
             max_cycles: int = 100, seed: int = 2000):
    """Cycles to 1e-6 of the mixed-precision solve on box images (the 2D
    deblurring right-hand sides) with the handle's weight set 0."""
    dev = torch.device("cuda:0")
    n = h.problem.n
    alpha = torch.full((batch,), alpha_value, dtype=torch.float64, device=dev)
    u = torch.tensor(np.stack([inputs.boxes_image(n, seed + i) for i in range(batch)]), device=dev)
    b = h.apply_operator(0, u, alpha, "fp64")
    try:
        _, cyc, hist, st = h.solve(b, alpha, rtol=1e-6, max_cycles=max_cycles, nu1=nu1, nu2=nu2,
                                   use_fprime=use_fprime, precision="mixed", history=True)
    except nmg.NMGError as e:
        return None, str(e)
    return cyc, st


def merge(argv):
    """``merge --out F --nu1 1 --nu2 1 --fprime a.npz:k b.npz:k ...``: one file
    holding the selected sets in the given order (alphas taken from each
    source file's metadata) plus the cycle the solver should run."""
    ap = argparse.ArgumentParser(prog="train_weights merge")
    ap.add_argument("--out", required=True)
    ap.add_argument("--nu1", type=int, default=1)
    ap.add_argument("--nu2", type=int, default=1)
    ap.add_argument("--fprime", action="store_true")
    ap.add_argument("sources", nargs="+")
    a = ap.parse_args(argv)
    sets, alphas, metas = [], [], []
    for src in a.sources:
        path, k = src.rsplit(":", 1)
        meta, ss = load_weights(path)
        sets.append(ss[int(k)])
        alphas.append(meta["alphas"][int(k)])
        metas.append({"file": os.path.basename(path), "set": int(k), **{x: meta.get(x) for x in
                      ("steps", "batch", "lr", "mask", "rollout", "precision", "seed", "use_fprime", "init")}})
    base = load_weights(a.sources[0].rsplit(":", 1)[0])[0]
    meta = dict(n=base["n"], s=base["s"], levels=base["levels"], channels=base["channels"], ksize=3,
                alphas=alphas, cycle={"nu1": a.nu1, "nu2": a.nu2, "use_fprime": bool(a.fprime)}, sources=metas)
    save_weights(a.out, meta, sets)
    print(f"wrote {a.out} with alphas {alphas}")


def coarsest_level_sweep(argv):
    """``levels --weights F [--set k] [--levels 2 3 4 5] [--batch 16]``: the
    coarsest-level change of Sec. 4 (loss ablation): smoothers trained with L
    levels solve with L' <= L levels (the first L'-1 smoothers, exact solve on
    level L'); prints the cycles to 1e-6 per L'.  A coarser L' needs a
    coarsest grid small enough for the dense factor."""
    ap = argparse.ArgumentParser(prog="train_weights levels")
    ap.add_argument("--weights", required=True)
    ap.add_argument("--set", type=int, default=0)
    ap.add_argument("--levels", type=int, nargs="+", default=None)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--max-cycles", type=int, default=200)
    a = ap.parse_args(argv)
    nmg.load_library()
    meta, sets = load_weights(a.weights)
    cyc_cfg = meta.get("cycle", {"nu1": 1, "nu2": 1, "use_fprime": False})
    alpha = meta["alphas"][a.set]
    out = {}
    for Lp in a.levels or list(range(2, meta["levels"] + 1)):
        if Lp > meta["levels"]:
            raise SystemExit(f"the weights have {meta['levels']} levels; L' = {Lp} is not available")
        prob = nmg.Problem(n=meta["n"], s=meta["s"], levels=Lp, max_batch=a.batch, channels=tuple(meta["channels"]),
                           ksize=meta.get("ksize", 3), operator=meta.get("operator", "normal"))
        try:
            h = nmg.setup_hierarchy(prob)
        except nmg.NMGError as e:
            print(f"L' = {Lp}: {e}", flush=True)
            continue
        for l in range(Lp - 1):
            h.load_smoother_weights(l, 0, [sets[a.set][l]])
        cyc, st = evaluate(h, alpha, a.batch, cyc_cfg["nu1"], cyc_cfg["nu2"], cyc_cfg["use_fprime"], a.max_cycles)
        h.close()
        if cyc is None:
            print(f"L' = {Lp}: {st}", flush=True)
            continue
        out[Lp] = (float(cyc.mean()), int(cyc.max()), int(st))
        print(f"L' = {Lp}: alpha {alpha:g} cycles mean {cyc.mean():.2f} max {cyc.max()} status {st}", flush=True)
    return out


def main(argv=None):
    import sys
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "merge":
        return merge(argv[1:])
    if argv and argv[0] == "levels":
        return coarsest_level_sweep(argv[1:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=255)
    ap.add_argument("--s", type=float, default=0.01)
    ap.add_argument("--levels", type=int, default=5)
    ap.add_argument("--channels", type=int, nargs="+", default=[1, 32, 32, 1])
    ap.add_argument("--alphas", type=float, nargs="+", default=[1e-2, 1e-3, 1e-4])
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--mask", default="ramp", choices=["ramp", "band", "cycle"],
                    help="level-wise spectral loss with the ramp or band mask, or the combined loss of the whole "
                         "cycle (eq. loss_1, all levels trained jointly)")
    ap.add_argument("--rollout", type=int, default=0, help="K of Algorithm 5: k ~ U{1..K} rollout cycles per sample")
    ap.add_argument("--rollout-rescale", action="store_true",
                    help="rescale rolled-out samples to unit RMS (not part of Algorithm 5)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "mixed"])
    ap.add_argument("--seed", type=int, default=7000)
    ap.add_argument("--out", required=True)
    ap.add_argument("--init", default=None, help="npz written by this script; its last set initialises training")
    ap.add_argument("--fprime", action="store_true", help="train with F' in the loss (eq. loss_2_modified)")
    ap.add_argument("--steps-per-alpha", type=int, nargs="+", default=None)
    ap.add_argument("--eval-max-cycles", type=int, default=100, help="cycle limit of the post-training evaluation")
    ap.add_argument("--fno", type=int, nargs=4, default=None, metavar=("C", "LAYERS", "MODES", "KSIZE"),
                    help="train FNO smoothers (width, Fourier layers, modes, convolution size) instead of the CNN")
    ap.add_argument("--operator", default="normal", choices=["normal", "kernel"],
                    help="fine operator: alpha I + K^T K (normal) or alpha I (x) I + K (x) K (kernel)")
    a = ap.parse_args(argv)
    nmg.load_library()
    prob = nmg.Problem(n=a.n, s=a.s, levels=a.levels, dim=2, max_batch=a.batch, channels=tuple(a.channels),
                       ksize=3, n_weight_sets=1, operator=a.operator, fno=tuple(a.fno) if a.fno else None)
    h = nmg.setup_hierarchy(prob)
    L = a.levels
    if a.init:
        _, init_sets = load_weights(a.init)
        for l in range(L - 1):
            h.load_smoother_weights(l, 0, [init_sets[-1][l]])
    elif a.fno:
        from .fno import pack_fno_weights
        for l in range(L - 1):
            h.load_smoother_weights(l, 0, [pack_fno_weights(inputs.fno_params(2, *a.fno, a.seed + 10 * l))])
    else:
        for l in range(L - 1):
            h.load_smoother_weights(l, 0, inputs.he_normal_weights(tuple(a.channels), 3, 2, a.seed + 10 * l))
    sets = []
    alphas = sorted(a.alphas, reverse=True)
    for k, av in enumerate(alphas):
        steps = a.steps_per_alpha[k] if a.steps_per_alpha else a.steps
        print(f"training alpha={av:g} ({steps} steps, batch {a.batch}, mask {a.mask}, fprime {a.fprime})", flush=True)
        train_set(h, av, steps, a.batch, a.lr, a.mask, a.seed + 1000 * k, a.rollout, precision=a.precision,
                  use_fprime=a.fprime, rollout_rescale=a.rollout_rescale)
        sets.append([h.get_smoother_weights(l) for l in range(L - 1)])
        for nu in ((1, 1), (2, 0), (1, 0)):
            cyc, st = evaluate(h, av, min(16, a.batch), nu[0], nu[1], a.fprime, a.eval_max_cycles)
            if cyc is None:
                print(f"  eval alpha={av:g} V{nu} fprime={a.fprime}: {st}", flush=True)
            else:
                print(f"  eval alpha={av:g} V{nu} fprime={a.fprime}: cycles mean {cyc.mean():.1f} max {cyc.max()} "
                      f"status {st}", flush=True)
    meta = dict(n=a.n, s=a.s, levels=L, channels=list(a.channels), ksize=3, alphas=alphas,
                steps=a.steps_per_alpha or [a.steps] * len(alphas), batch=a.batch, lr=a.lr, mask=a.mask,
                rollout=a.rollout, rollout_rescale=bool(a.rollout_rescale), precision=a.precision, seed=a.seed, use_fprime=bool(a.fprime), init=a.init,
                operator=a.operator, fno=list(a.fno) if a.fno else None)
    save_weights(a.out, meta, sets)
    print(f"wrote {a.out}", flush=True)
    h.close()


if __name__ == "__main__":
    main()
