"""Benchmark: V-cycle solves/s to 1e-6 relative residual on 255x255 (256^2
cells) with a batch of 64 right-hand sides, plus p50/p99 solve latency.

One step = one batched solve of 64 synthetic deblurring problems
b = A u* (u* = 20 random boxes + N(0, 0.01) noise, alpha per right-hand side
drawn from {1e-2, 1e-3, 1e-4}) to relative residual 1e-6 with the
mixed-precision neural V-cycle (BF16 MFMA smoother, FP32 cycle, FP64
refinement and coarse Cholesky).  Inputs of every step are resident on the
GPU before the timed region starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "V-cycle solves/s to 1e-6 rel. residual, 256^2 batch 64; p50/p99 solve latency"
N, S, LEVELS, BATCH = 255, 0.01, 5, 64
CHANNELS = (1, 32, 32, 1)
ALPHAS = (1e-2, 1e-3, 1e-4)
PROFILE_PERIOD = 8  # the smoother roofline times every 8th solve iteration
FLOP_PER_PX = 2 * 9 * (1 * 32 + 32 * 32 + 32 * 1)  # 19,584: three 3x3 layers
# smoother input plane read + output plane written (FP32), plus a read of the
# output when it accumulates into x (no F')
PLANE_BYTES = 4 * N * N
BF16_PEAK_TFLOPS = 2500.0
FP32_VALU_PEAK_TFLOPS = 78.6  # non-packed FP32 FMA: 256 CUs x 64 lanes x 2 x 2.4 GHz
FP64_VALU_PEAK_TFLOPS = 78.6  # FP64 FMA at the same rate
FP32_MFMA_PEAK_TFLOPS = 157.3  # dense FP32 matrix (v_mfma_f32_16x16x4f32)
WEIGHTS = os.path.join(ROOT, "paper_2603_01064_amd", "weights", "grid255_s0.01.npz")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "smoother_mfma_grid255_b64_pmc.txt")
SMOOTHER_SRC = os.path.join(ROOT, "paper_2603_01064_amd", "csrc", "mfma_smoother.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_per_image():
    """Measured HBM bytes per (image x launch) of the level-1 smoother from the
    committed rocprofv3 counter summary, or None when it is missing or was
    taken on another version of the kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    txt = open(PMC_SUMMARY).read()
    want = source_hash(SMOOTHER_SRC)
    if f"kernel_source_sha256_16: {want}" not in txt:
        return None
    for line in txt.splitlines():
        if line.startswith("hbm_bytes_per_image:"):
            return float(line.split(":")[1])
    return None


def smoother_bytes_per_image(use_fprime):
    """Algorithmic HBM bytes of one level-1 smoother application to one image:
    the FP32 input plane is read; with F' next, the output is the zero-padded
    (N + 1)^2 BF16 plane that the F' kernel reads, else the FP32 plane
    x + S(r), read and written."""
    if use_fprime:
        return PLANE_BYTES + 2 * (N + 1) * (N + 1)
    return 3 * PLANE_BYTES


def bf16_errors(h, batch, cyc_cfg):
    """The BF16 error of the timed configuration, measured against the
    library's own FP64 path (whose parity with the oracle the tests fix at
    1e-12) on one batch of 64 right-hand sides:
      * smoother: ||S_bf16(v) - S_fp64(v)|| / ||S_fp64(v)|| on level 1 for
        i.i.d. N(0, 1) inputs v and for the right-hand sides themselves (whose
        smooth content the network largely cancels, so that the BF16 rounding
        of its activations is large against its small output), and
      * cycle: one V-cycle from zero, ||A (x_mixed - x_fp64)|| / ||y||, the
        difference seen through the operator (x itself carries components that
        the cycle amplifies by up to 1/alpha, which the residual does not).
    Maxima and means per alpha."""
    import torch
    alpha, ws, b, _ = batch
    al = alpha.cpu().numpy()
    h.prepare(alpha)
    s64 = h.apply_smoother(0, b, alpha, weight_set=ws, precision="fp64")
    s16 = h.apply_smoother(0, b.float(), alpha, weight_set=ws, precision="mixed").double()
    e_sm = ((s16 - s64).flatten(1).norm(dim=1) / s64.flatten(1).norm(dim=1)).cpu().numpy()
    # the same on i.i.d. N(0, 1) inputs (the smoother's own accuracy, without
    # the cancellation that a smooth right-hand side brings into its output)
    g = torch.Generator(device=b.device).manual_seed(5)
    z = torch.randn(b.shape, dtype=torch.float64, device=b.device, generator=g)
    z64 = h.apply_smoother(0, z, alpha, weight_set=ws, precision="fp64")
    z16 = h.apply_smoother(0, z.float(), alpha, weight_set=ws, precision="mixed").double()
    e_rn = ((z16 - z64).flatten(1).norm(dim=1) / z64.flatten(1).norm(dim=1)).cpu().numpy()
    kw = dict(weight_set=ws, nu1=cyc_cfg["nu1"], nu2=cyc_cfg["nu2"], use_fprime=cyc_cfg["use_fprime"])
    x64 = h.vcycle(b, torch.zeros_like(b), alpha, precision="fp64", **kw)
    x16 = h.vcycle(b.float(), torch.zeros_like(b, dtype=torch.float32), alpha, precision="mixed", **kw).double()
    d = h.apply_operator(0, (x16 - x64).contiguous(), alpha, "fp64")
    e_cy = (d.flatten(1).norm(dim=1) / b.flatten(1).norm(dim=1)).cpu().numpy()
    out = {"reference": "library FP64 path on the same inputs and weights", "rhs": int(len(al))}
    for name, e in (("smoother_rel_random_input", e_rn), ("smoother_rel_rhs_input", e_sm),
                    ("vcycle_operator_rel", e_cy)):
        out[name] = {f"{av:g}": {"max": float(f"{e[np.isclose(al, av)].max():.3e}"),
                                 "mean": float(f"{e[np.isclose(al, av)].mean():.3e}")}
                     for av in ALPHAS if np.isclose(al, av).any()}
    return out


def make_inputs(steps, seed0=20000):
    from paper_2603_01064_amd import inputs
    out = []
    for k in range(steps):
        alpha = inputs.alpha_mix(BATCH, seed0 + k)
        u = np.stack([inputs.boxes_image(N, 2000 + 1000 * k + i) for i in range(BATCH)])
        out.append((alpha, u))
    return out


def split_layers(flat, channels=CHANNELS, k=3):
    """Per-layer [Cout][Cin][k][k] views of one level's flat weight vector."""
    out, off = [], 0
    for cin, cout in zip(channels[:-1], channels[1:]):
        size = cout * cin * k * k
        out.append(np.asarray(flat[off:off + size], dtype=np.float64).reshape(cout, cin, k, k))
        off += size
    return out


def cpu_baseline(meta, sets, host_batch, budget_s=20.0, max_cycles=200):
    """The FP64 oracle solving right-hand sides of the benchmark's first timed
    batch to the same 1e-6 relative residual with the same trained weight
    sets and cycle, one right-hand side at a time on the host's cores (torch
    intra-op threads = the cores this process may run on).  Right-hand sides
    are taken round-robin over the three alphas until `budget_s` is spent (at
    least one per alpha).  Measured solves/s = solves / wall time."""
    import torch

    import oracle as O
    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    alpha_np, u = host_batch
    set_alphas = meta["alphas"]
    H = O.build_hierarchy(N, S, LEVELS, dim=2)
    smoothers = {}
    nu1, nu2, fp = meta["cycle"]["nu1"], meta["cycle"]["nu2"], meta["cycle"]["use_fprime"]
    tag = f"V({nu1},{nu2})" + ("+F'" if fp else "")
    by_alpha = {}
    for i, v in enumerate(alpha_np):
        by_alpha.setdefault(float(v), []).append(i)
    order = []
    for j in range(max(len(v) for v in by_alpha.values())):
        for av in sorted(by_alpha):
            if j < len(by_alpha[av]):
                order.append(by_alpha[av][j])
    t0 = time.perf_counter()
    done = []
    for i in order:
        av = float(alpha_np[i])
        k = set_alphas.index(min(set_alphas, key=lambda s_: abs(math.log(s_ / av))))
        if k not in smoothers:
            smoothers[k] = [O.neural_smoother([torch.tensor(w) for w in split_layers(sets[k][l])], 2)
                            for l in range(LEVELS - 1)]
        alpha = torch.tensor([av], dtype=torch.float64)
        y = O.apply_operator(H, 0, torch.tensor(u[i]).unsqueeze(0), alpha)
        r = O.solve(H, smoothers[k], y, alpha, tol=1e-6, max_cycles=max_cycles, nu1=nu1, nu2=nu2, use_fprime=fp)
        done.append((av, int(r.cycles[0]), bool(r.converged[0])))
        if time.perf_counter() - t0 > budget_s and len(done) >= len(by_alpha):
            break
    total = time.perf_counter() - t0
    cyc_by = {f"{av:g}": [c for a_, c, _ in done if a_ == av] for av in sorted(by_alpha)}
    return {
        "value": round(len(done) / total, 4),
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{len(done)} right-hand sides of the first timed batch (round-robin over the alphas), each "
                  f"solved to 1e-6 by the FP64 oracle's {tag} iteration with its trained weight set, in "
                  f"{total:.1f} s on {cores} threads; cycles per alpha {cyc_by}; converged "
                  f"{sum(c for _, _, c in done)}/{len(done)}",
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--weights", default=WEIGHTS)
    ap.add_argument("--max-cycles", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serial-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the continuous-batching measurements")
    ap.add_argument("--no-training", action="store_true", help="skip the training-step measurement")
    ap.add_argument("--no-mixed-sizes", action="store_true",
                    help="skip the serving stream over grid sides 64..1024 (needs the s = 2.5h weights)")
    ap.add_argument("--mixed-requests", type=int, default=300, help="requests per arrival rate, mixed sizes")
    ap.add_argument("--no-large", action="store_true", help="skip the 2047x2047 batch-16 solve")
    ap.add_argument("--no-fno", action="store_true", help="skip the FNO smoother kernel timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 64 MiB device copy before timing (reference kernel for HBM counters)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {a.gpus}); every right-hand side is "
              f"independent, see the sharding notes in DESIGN.md", file=sys.stderr)
        return 2

    import torch

    from paper_2603_01064_amd import nmg
    from paper_2603_01064_amd.train_weights import load_weights

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    nmg.load_library()
    meta, sets = load_weights(a.weights)
    assert meta["n"] == N and abs(meta["s"] - S) < 1e-12 and meta["levels"] == LEVELS
    cyc_cfg = meta.get("cycle", {"nu1": 1, "nu2": 1, "use_fprime": bool(meta.get("use_fprime", False))})
    meta["cycle"] = cyc_cfg
    set_alphas = list(meta["alphas"])
    h = nmg.setup_hierarchy(nmg.Problem(n=N, s=S, levels=LEVELS, max_batch=BATCH, channels=CHANNELS, ksize=3,
                                        n_weight_sets=len(sets)))
    for k, ws in enumerate(sets):
        for l in range(LEVELS - 1):
            h.load_smoother_weights(l, k, [ws[l]])

    # ---- inputs, resident on the GPU before timing
    log(f"generating {a.warmup + a.steps} batches of {BATCH} right-hand sides")
    host = make_inputs(a.warmup + a.steps)
    batches = []
    for alpha_np, u in host:
        alpha = torch.tensor(alpha_np, dtype=torch.float64, device=dev)
        ws = torch.tensor([set_alphas.index(min(set_alphas, key=lambda s: abs(math.log(s / v)))) for v in alpha_np],
                          dtype=torch.int32, device=dev)
        b = h.apply_operator(0, torch.tensor(u, device=dev), alpha, "fp64")
        batches.append((alpha, ws, b, torch.empty_like(b)))
    torch.cuda.synchronize()

    def run(batch):
        alpha, ws, b, x = batch
        done = np.full(BATCH, -1.0)
        _, cyc, _, st = h.solve(b, alpha, weight_set=ws, rtol=1e-6, max_cycles=a.max_cycles, nu1=cyc_cfg["nu1"],
                                nu2=cyc_cfg["nu2"], use_fprime=cyc_cfg["use_fprime"], precision="mixed", x=x,
                                done_ms=done)
        return cyc, done, st

    # warm-up with the timing of the timed region switched on, so that the
    # iteration graphs of both kinds (with and without the timing launches)
    # are captured before it
    h.profile_levels([0])
    h.profile_sample(PROFILE_PERIOD)
    h.profile_enable(("smoother",))
    for k in range(a.warmup):
        log(f"warmup {k + 1}/{a.warmup}")
        run(batches[k])
    h.profile_enable(())
    if a.copy_calibration:
        src = torch.ones(16 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # ---- timed region (the level-1 smoother is timed on every PROFILE_PERIOD-th
    # solve iteration; the others replay graphs without timing launches)
    h.profile_levels([0])
    h.profile_sample(PROFILE_PERIOD)
    h.profile_enable(("smoother",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles, lat, status = [], [], []
    for k in range(a.steps):
        cyc, done, st = run(batches[a.warmup + k])
        cycles.append(cyc)
        lat.append(done)
        status.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sm_ms, sm_n = h.profile_query("smoother", 0)
    rhs_timed = h.profile_rhs()
    h.profile_enable(())
    h.profile_sample(1)
    log(f"timed {a.steps} steps in {elapsed:.3f} s")
    cycles = np.concatenate(cycles)
    lat = np.concatenate(lat)
    alphas_all = np.concatenate([host[a.warmup + k][0] for k in range(a.steps)])
    converged = lat >= 0
    value = BATCH * a.steps / elapsed
    by_alpha = {f"{av:g}": float(cycles[np.isclose(alphas_all, av)].mean()) for av in ALPHAS
                if np.isclose(alphas_all, av).any()}
    # Converged right-hand sides leave the batch, so level-1 smoother launches
    # process between 1 and 64 images; nu1 + nu2 launches per timed iteration
    # of each right-hand side still iterating give the images of the timed launches.
    images = (cyc_cfg["nu1"] + cyc_cfg["nu2"]) * rhs_timed
    avg_ms = sm_ms / max(sm_n, 1)
    mean_images = images / max(sm_n, 1)
    achieved = FLOP_PER_PX * N * N * images / (sm_ms * 1e-3) / 1e12 if sm_ms > 0 else 0.0
    tpi = traffic_per_image()
    roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
            "traffic": round(tpi * mean_images) if tpi is not None else None,
            "kernel": "k_smoother_mfma<3> on level 1 (255x255, BF16 CNN 1-32-32-1)",
            "avg_launch_ms": round(avg_ms, 4), "launches": sm_n, "images_per_launch": round(mean_images, 2),
            "timed_iterations": f"every {PROFILE_PERIOD}th solve iteration of the timed region",
            "flop_per_launch": round(FLOP_PER_PX * N * N * mean_images),
            "algorithmic_bytes_per_launch": round(smoother_bytes_per_image(cyc_cfg["use_fprime"]) * mean_images)}
    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(1e3 * elapsed / a.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {
            "workload": "2D deblurring solve, 255x255 unknowns (256^2 cells), Gaussian s=0.01 truncated at 4s, "
                        "alpha per RHS in {1e-2,1e-3,1e-4}, 5 levels to 15x15, CNN 1-32-32-1 3x3 smoothers, "
                        "batch 64, rtol 1e-6",
            "global_batch": BATCH, "grid": N, "levels": LEVELS,
            "cycle": f"V({cyc_cfg['nu1']},{cyc_cfg['nu2']})" + ("+F'" if cyc_cfg["use_fprime"] else ""),
            "precision": "BF16 smoother on MFMA (FP32 accumulate), FP32 cycle, FP64 refinement + coarse Cholesky",
            "p50_ms": round(float(np.percentile(lat[converged], 50)), 3) if converged.any() else None,
            "p99_ms": round(float(np.percentile(lat[converged], 99)), 3) if converged.any() else None,
            "mean_cycles": round(float(cycles.mean()), 2), "cycles_by_alpha": by_alpha,
            "converged": int(converged.sum()), "solves": int(len(lat)),
        },
        "roofline": roof,
    }
    log("BF16 error against the FP64 path (one batch)")
    res["bf16_error"] = bf16_errors(h, batches[a.warmup], cyc_cfg)
    log("stencil and transfer kernels: one profiled batch")
    res["roofline_stencil"] = stencil_roofline(h, run, batches[a.warmup + a.steps - 1])
    if not a.no_serial_baseline:
        res["serial_fp32_gpu"] = serial_fp32(nmg, sets, set_alphas, cyc_cfg, host[a.warmup][0], host[a.warmup][1],
                                             a.max_cycles)
        if res["serial_fp32_gpu"]["value"] > 0:
            res["serial_fp32_gpu"]["speedup_solves_per_s"] = round(value / res["serial_fp32_gpu"]["value"], 1)
            if res["config"]["p99_ms"] and res["serial_fp32_gpu"]["p99_ms"]:
                res["serial_fp32_gpu"]["p99_ratio"] = round(res["serial_fp32_gpu"]["p99_ms"] / res["config"]["p99_ms"], 2)
    if not a.no_training:
        log("training step (127x127, batch 256)")
        res["training"] = training(nmg)
    if not a.no_serving:
        log("serving: continuous batching on Poisson arrivals")
        res["serving"] = serving(nmg, h, sets, set_alphas, cyc_cfg, batches[a.warmup:], a.max_cycles,
                                 serial=not a.no_serial_baseline)
    if not a.no_fno:
        log("FNO smoother kernel timing (255x255, C=64, 5 layers)")
        res["fno_smoother"] = fno_smoother_timing(nmg)
    if not a.no_large and os.path.exists(LARGE_WEIGHTS):
        log("large solve: 2047x2047, batch 16")
        res["large_solve"] = large_solve(nmg)
    if not a.no_mixed_sizes and os.path.exists(MIXED_WEIGHTS):
        log("serving: grid sides 64..1024 through one pool")
        res["serving_mixed_sizes"] = mixed_sizes_serving(nmg, count=a.mixed_requests, max_cycles=a.max_cycles,
                                                         serial=not a.no_serial_baseline)
    if not a.no_cpu_baseline:
        log("timing the CPU oracle")
        res["cpu_baseline"] = cpu_baseline(meta, sets, host[a.warmup])
    print(json.dumps(res), flush=True)
    h.close()
    return 0


HBM_PEAK_GBS = 8000.0


def stencil_roofline(h, run, batch):
    """Achieved rates of the level-1 stencil and transfer kernels, timed by the
    library profiler (device clock stamps around each launch inside the
    captured iterations) on one more batch after the timed region, so the
    headline timing carries no extra stamps.  Algorithmic bytes count each
    input read once and each output written once; only right-hand sides still
    iterating count (launches also cover padding slots of a launch size)."""
    import torch
    kinds = ("operator", "restrict", "prolong", "refine")
    h.profile_levels([0])
    h.profile_enable(kinds)
    torch.cuda.synchronize()
    cyc, _, _ = run(batch)
    torch.cuda.synchronize()
    rhs_cycles = int(cyc.sum())
    px, pc = N * N, ((N - 1) // 2) ** 2
    flop_res = 2 * 2 * 41 + 3  # two 41-tap axis passes (G radius 20) plus the alpha term and the subtraction
    rows = {
        # kind: (launches per right-hand-side cycle, bytes per image, flop per image, label, bound)
        "operator": (2, 12 * px, flop_res * px, "FP32 residual y - A x, level 1 (k_residual_fixed)", "alu"),
        "restrict": (1, 4 * px + 4 * pc, 0, "full-weighting restriction, level 1 -> 2 (k_restrict)", "hbm"),
        "prolong": (1, 4 * pc + 8 * px, 0, "interpolation and correction, level 2 -> 1 (k_prolong_add)", "hbm"),
        "refine": (1, 36 * px, (flop_res + 2) * px,
                   "FP64 refinement residual with the fused update (k_rows_fixed + k_cols_fixed + k_sumsq_final)",
                   "hbm"),
    }
    out = {}
    for kind, (per_cycle, bpi, fpi, label, bound) in rows.items():
        ms, n = h.profile_query(kind, 0)
        images = per_cycle * rhs_cycles
        if n == 0 or ms <= 0:
            continue
        gbs = bpi * images / (ms * 1e-3) / 1e9
        e = {"kernel": label, "bound": bound, "launches": n, "avg_launch_ms": round(ms / n, 4),
             "images_per_launch": round(images / n, 2), "algorithmic_bytes_per_launch": round(bpi * images / n),
             "achieved_gbs": round(gbs, 1), "hbm_peak_gbs": HBM_PEAK_GBS, "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        if fpi:
            tf = fpi * images / (ms * 1e-3) / 1e12
            peak = FP32_VALU_PEAK_TFLOPS if kind == "operator" else FP64_VALU_PEAK_TFLOPS
            e.update({"achieved_tflops": round(tf, 2), "valu_peak_tflops": peak, "valu_frac": round(tf / peak, 4)})
        out[kind] = e
    h.profile_enable(())
    h.profile_levels(None)
    return out


def training(nmg, steps=10, warmup=2):
    """Level-wise training step (loss, hand-written adjoint, Adam) at the
    training workload's shape: 127x127, s = 0.01, five levels, CNN 1-32-32-1,
    batch 256 of i.i.d. N(0, 1) error vectors, alpha 1e-3, band mask, FP32 with
    BF16 MFMA forward, lr 1e-3."""
    import torch

    from paper_2603_01064_amd import inputs
    dev = torch.device("cuda:0")
    n, s, L, B = 127, 0.01, 5, 256
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, max_batch=B, channels=CHANNELS, ksize=3))
    for l in range(L - 1):
        h.load_smoother_weights(l, 0, inputs.he_normal_weights(CHANNELS, 3, 2, 7000 + 10 * l))
    alpha = torch.full((B,), 1e-3, dtype=torch.float64, device=dev)
    es = [torch.tensor(inputs.iid_normal((B, n, n), 40000 + k), dtype=torch.float32, device=dev)
          for k in range(warmup + steps)]
    for k in range(warmup):
        h.train_step(es[k], alpha, mask="band", precision="mixed", lr=1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    first = last = None
    for k in range(steps):
        losses = h.train_step(es[warmup + k], alpha, mask="band", precision="mixed", lr=1e-3)
        first = float(losses.sum()) if first is None else first
        last = float(losses.sum())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h.close()
    # algorithmic network work per step: forward plus backward (data and weight
    # gradients, 2x the forward) of each level's smoother on its level, for
    # the batch; the loss transforms, transfers and the activation recompute
    # are not counted
    px = sum((((n + 1) >> l) - 1) ** 2 for l in range(L - 1))
    flop = 3 * FLOP_PER_PX * px * B
    tflops = flop / (dt / steps) / 1e12
    return {"ms_per_step": round(1e3 * dt / steps, 2), "samples_per_s": round(B * steps / dt, 1), "steps": steps,
            "batch": B, "grid": n, "levels": L, "mask": "band", "loss_sum_first": first, "loss_sum_last": last,
            "network_gflop_per_step": round(flop / 1e9, 1), "achieved_tflops": round(tflops, 2),
            "mfma_frac": round(tflops / BF16_PEAK_TFLOPS, 4),
            "flop_note": "3 x 19,584 FLOP per pixel (forward + backward of the CNN 1-32-32-1) on levels "
                         "127^2, 63^2, 31^2, 15^2, batch 256; against the dense BF16 MFMA peak"}


def _serial_handle(nmg, sets):
    h1 = nmg.setup_hierarchy(nmg.Problem(n=N, s=S, levels=LEVELS, max_batch=1, channels=CHANNELS, ksize=3,
                                         n_weight_sets=len(sets)))
    for k, ws in enumerate(sets):
        for l in range(LEVELS - 1):
            h1.load_smoother_weights(l, k, [ws[l]])
    return h1


def serial_fp32(nmg, sets, set_alphas, cyc_cfg, alpha_np, u, max_cycles, count=8):
    """Plain FP32 V-cycle solving one right-hand side at a time (no batching,
    no BF16, no refinement) on the first `count` problems of a batch, with the
    tiled FP32 smoother and captured iteration graphs (one warm-up solve
    captures them first)."""
    import torch
    dev = torch.device("cuda:0")
    h1 = _serial_handle(nmg, sets)
    probs = []
    for i in range(count):
        alpha = torch.tensor([alpha_np[i]], dtype=torch.float64, device=dev)
        wsi = set_alphas.index(min(set_alphas, key=lambda s: abs(math.log(s / alpha_np[i]))))
        ws = torch.tensor([wsi], dtype=torch.int32, device=dev)
        b = h1.apply_operator(0, torch.tensor(u[i:i + 1], device=dev), alpha, "fp64")
        probs.append((alpha, ws, b))
    a0, w0, b0 = probs[0]
    h1.solve(b0, a0, weight_set=w0, rtol=1e-6, max_cycles=2, nu1=cyc_cfg["nu1"], nu2=cyc_cfg["nu2"],
             use_fprime=cyc_cfg["use_fprime"], precision="fp32")  # graph capture, coarse factors
    torch.cuda.synchronize()
    lat, cyc_all, ok = [], [], 0
    t0 = time.perf_counter()
    for alpha, ws, b in probs:
        t1 = time.perf_counter()
        try:
            _, cyc, _, st = h1.solve(b, alpha, weight_set=ws, rtol=1e-6, max_cycles=max_cycles,
                                     nu1=cyc_cfg["nu1"], nu2=cyc_cfg["nu2"], use_fprime=cyc_cfg["use_fprime"],
                                     precision="fp32")
            ok += int(st == 0)
            cyc_all.append(int(cyc[0]))
        except nmg.NMGError:
            cyc_all.append(-1)
        lat.append(1e3 * (time.perf_counter() - t1))
    elapsed = time.perf_counter() - t0
    h1.close()
    return {"value": round(count / elapsed, 3), "unit": "solves/s", "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2), "converged": ok, "solves": count, "cycles": cyc_all,
            "note": "one request at a time, plain FP32 cycle, tiled FP32 convolution smoother, captured graphs"}


def serving(nmg, h, sets, set_alphas, cyc_cfg, batches, max_cycles, rates=(20.0, 1000.0), low_count=48,
            serial=True):
    """Continuous batching through the handle's 64 slots on Poisson arrival
    traces of the same synthetic requests (latency = arrival to completion,
    queueing included), and the serial plain-FP32 solver on the low-rate
    trace; plus the saturated rate with every request queued at once."""
    import torch

    from paper_2603_01064_amd import inputs
    from paper_2603_01064_amd.serve import serve_requests, serve_serially
    b = torch.cat([bt[2] for bt in batches])
    alpha = torch.cat([bt[0] for bt in batches]).cpu().numpy()
    ws = torch.cat([bt[1] for bt in batches]).cpu().numpy()
    x = torch.empty_like(b)
    kw = dict(rtol=1e-6, max_cycles=max_cycles, nu1=cyc_cfg["nu1"], nu2=cyc_cfg["nu2"],
              use_fprime=cyc_cfg["use_fprime"], precision="mixed")
    out = {}
    total = b.shape[0]
    rep = serve_requests(h, b, x, alpha, ws, np.zeros(total), **kw)
    out["saturated"] = rep.summary()
    for rate in rates:
        cnt = low_count if rate < 100 else total
        arr = inputs.poisson_arrivals(rate, cnt, seed=31000 + int(rate))
        arr = arr - arr[0]
        rep = serve_requests(h, b[:cnt], x[:cnt], alpha[:cnt], ws[:cnt], arr, **kw)
        out[f"poisson_{int(rate)}_per_s"] = rep.summary()
        if serial and rate < 100:
            h1 = _serial_handle(nmg, sets)
            dev = b.device

            def solve_one(i):
                try:
                    _, cyc, _, st = h1.solve(b[i:i + 1], torch.tensor([alpha[i]], dtype=torch.float64, device=dev),
                                             weight_set=torch.tensor([int(ws[i])], dtype=torch.int32, device=dev),
                                             rtol=1e-6, max_cycles=max_cycles, nu1=cyc_cfg["nu1"],
                                             nu2=cyc_cfg["nu2"], use_fprime=cyc_cfg["use_fprime"], precision="fp32")
                    return int(cyc[0]), int(st)
                except nmg.NMGError:
                    return -1, -1

            solve_one(0)  # graph capture and coarse factors before the trace
            srep = serve_serially(solve_one, arr)
            h1.close()
            out[f"poisson_{int(rate)}_per_s"]["serial_fp32"] = srep.summary()
    return out


LARGE_WEIGHTS = os.path.join(ROOT, "paper_2603_01064_amd", "weights", "grid255_s10.24h_c4.npz")


def large_solve(nmg, batch=16, max_cycles=400):
    """2047^2 unknowns (2048^2 cells), s = 0.005 (s/h = 10.24, band radius 80
    of G_1), alpha = 1e-4, 16 right-hand sides b = sum of 500 Gaussian blobs,
    eight levels down to 15^2 with the dense FP64 Cholesky solve there.  The
    CNN 1-32-32-32-1 smoothers are trained per level at 255^2 (s/h = 10.24,
    5.12, 2.56, 1.28 on levels 1-4); levels 5-7 (s/h = 0.64, 0.32, 0.16, where
    the Gaussian is narrower than the grid spacing) use the weighted Jacobi
    smoother of Sec. 2.2 with omega = 0.8.  Times the batched mixed solve to
    relative residual 1e-6 and continued to 1e-14 (its error against the exact
    solution, below 1e-10, is checked by the large-solve tests), and the plain
    FP32 cycle, which cannot resolve 1e-6 on this operator, for its time per
    cycle and the residual it reaches."""
    import torch

    from paper_2603_01064_amd import inputs
    from paper_2603_01064_amd.train_weights import load_weights
    dev = torch.device("cuda:0")
    meta, sets = load_weights(LARGE_WEIGHTS)
    n, s, L, alpha_v, omega = 2047, 0.005, 8, 1e-4, 0.8
    k = meta["alphas"].index(min(meta["alphas"], key=lambda v: abs(math.log(v / alpha_v))))
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, max_batch=batch, channels=tuple(meta["channels"]),
                                        ksize=3, n_weight_sets=1))
    trained = meta["levels"] - 1  # smoothing levels of the training hierarchy
    for l in range(L - 1):
        if l < trained:
            h.load_smoother_weights(l, 0, [sets[k][l]])
        else:
            h.set_jacobi_smoother(l, omega)
    cyc = meta["cycle"]
    b = torch.tensor(np.stack([inputs.blobs_image(n, 44000 + i) for i in range(batch)]), device=dev)
    alpha = torch.full((batch,), alpha_v, dtype=torch.float64, device=dev)
    out = {"workload": "2047x2047 unknowns, s=0.005 (s/h=10.24), alpha 1e-4, 8 levels to 15x15 (FP64 Cholesky), "
                       "batch 16, b = 500 Gaussian blobs (widths U(2,20) px)",
           "smoothers": f"levels 1-{trained}: CNN 1-32-32-32-1 3x3 trained at 255^2 with s/h = 10.24 "
                        f"(alpha {meta['alphas'][k]:g}); levels {trained + 1}-{L - 1}: weighted Jacobi, "
                        f"omega {omega}"}
    x = torch.empty_like(b)
    kw = dict(nu1=cyc["nu1"], nu2=cyc["nu2"], use_fprime=cyc["use_fprime"])
    h.solve(b[:1], alpha[:1], rtol=1e-6, max_cycles=max_cycles, precision="mixed", **kw)  # capture, factors
    # the plain FP32 cycle (tiled FP32 convolution smoother, FP32 residuals) stalls near 2e-5 on this
    # operator, so it runs 3 cycles for its per-cycle time
    for prec, rtol, cap in (("mixed", 1e-6, max_cycles), ("fp32", 1e-6, 3), ("mixed", 1e-14, max_cycles)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, cycles, hist, st = h.solve(b, alpha, rtol=rtol, max_cycles=cap, precision=prec, x=x,
                                      history=True, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = b - h.apply_operator(0, x, alpha, "fp64")
        rel = (r.flatten(1).norm(dim=1) / b.flatten(1).norm(dim=1)).cpu().numpy()
        key = f"{prec}_to_{rtol:g}"
        out[key] = {"seconds": round(dt, 3), "solves_per_s": round(batch / dt, 3), "status": int(st),
                    "max_cycles": cap, "ms_per_cycle": round(1e3 * dt / max(1, int(np.max(cycles))), 1),
                    "cycles_mean": round(float(np.mean(cycles)), 2), "cycles_max": int(np.max(cycles)),
                    "max_rel_residual_fp64": float(rel.max())}
        log(f"2047^2 {prec} to {rtol:g}: {dt:.2f} s, cycles {np.mean(cycles):.1f}, max residual {rel.max():.2e}")
    h.close()
    return out


def fno_smoother_timing(nmg, batch=8, reps=3):
    """One application of the FNO smoother (the appendix's 2D network for
    h = 1/256: C = 64, 5 Fourier layers, k = 32 modes, 5x5 convolution) to
    `batch` right-hand sides of 255^2, FP32, seeded weights (a kernel timing:
    no trained FNO weights ship).  Algorithmic FLOPs per image: the
    convolutions 2 C^2 ks^2 n^2 per layer plus lift, projection, the
    truncated DFTs (4 n^2 2k + 8 n (2k) k per channel and direction) and the
    mode mixing 8 C^2 (2 k^2)."""
    import torch

    from paper_2603_01064_amd import inputs
    from paper_2603_01064_amd.fno import pack_fno_weights
    dev = torch.device("cuda:0")
    n, C, NL, k, ks = 255, 64, 5, 32, 5
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=0.01, levels=2, max_batch=batch, fno=(C, NL, k, ks)))
    h.load_smoother_weights(0, 0, [pack_fno_weights(inputs.fno_params(2, C, NL, k, ks, 47000))])
    b = torch.randn(batch, n, n, dtype=torch.float32, device=dev)
    alpha = torch.full((batch,), 1e-3, dtype=torch.float64, device=dev)
    h.apply_smoother(0, b, alpha, precision="fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        h.apply_smoother(0, b, alpha, precision="fp32")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    h.close()
    px = n * n
    per_layer = 2 * C * C * ks * ks * px + C * (4 * px * 2 * k + 8 * n * 2 * k * k) * 2 + 8 * C * C * 2 * k * k
    flop = batch * (NL * per_layer + 4 * C * px)
    tf = flop / dt / 1e12
    return {"workload": f"FNO smoother, 255x255, C={C}, {NL} Fourier layers, k={k}, ks={ks}, batch {batch}, FP32",
            "ms_per_application": round(1e3 * dt, 2), "gflop_per_application": round(flop / 1e9, 1),
            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / FP32_MFMA_PEAK_TFLOPS, 4),
                         "note": "whole application: the layer convolutions (83% of the FLOPs) on the FP32 MFMA, "
                                 "the truncated transforms and mode mixing on the VALU; against the dense FP32 "
                                 "MFMA peak"}}


MIXED_WEIGHTS = os.path.join(ROOT, "paper_2603_01064_amd", "weights", "grid255_s2.5h.npz")
MIXED_SIDES = (64, 128, 256, 512, 1024)
MIXED_SLOTS = {64: 64, 128: 64, 256: 64, 512: 32, 1024: 16}


def _mixed_handle(nmg, side, meta, sets, max_batch):
    """Grid side N (N - 1 interior points per axis), s = 2.5 / N, levels down
    to 15^2.  Level l uses trained level min(l, deepest): the kernel width in
    grid units (s/h = 2.5) and so every level's operator matches the training
    grid's level l up to boundary rows; deeper levels reuse the deepest set."""
    n = side - 1
    L = int(round(math.log2(side / 16))) + 1
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=2.5 / side, levels=L, max_batch=max_batch,
                                        channels=tuple(meta["channels"]), ksize=3, n_weight_sets=len(sets)))
    deepest = meta["levels"] - 2
    for k, ws in enumerate(sets):
        for l in range(L - 1):
            h.load_smoother_weights(l, k, [ws[min(l, deepest)]])
    return h


def mixed_sizes_serving(nmg, rates=(50.0, 100.0, 200.0, 400.0), count=300, serial_count=40, max_cycles=200,
                        budget=2 << 30, serial=True):
    """Serving stream of 2D solves with grid side uniform over 64..1024,
    s = 2.5 grid spacings, alpha log-uniform in [1e-5, 1e-2], box-image
    right-hand sides and Poisson arrivals, through one pool (one handle per
    side, 2 GiB budget) with the BF16/FP32/FP64 cycle to 1e-6 (weight set
    per request by `select_set`); the serial
    plain-FP32 one-request-at-a-time solver runs the first requests of the
    lowest-rate trace."""
    import torch

    from paper_2603_01064_amd import inputs
    from paper_2603_01064_amd.serve import serve_pool_requests, serve_serially
    from paper_2603_01064_amd.train_weights import load_weights, select_set
    dev = torch.device("cuda:0")
    meta, sets = load_weights(MIXED_WEIGHTS)
    set_alphas = list(meta["alphas"])
    cyc_cfg = meta["cycle"]
    kw = dict(rtol=1e-6, max_cycles=max_cycles, nu1=cyc_cfg["nu1"], nu2=cyc_cfg["nu2"],
              use_fprime=cyc_cfg["use_fprime"])
    handles = [_mixed_handle(nmg, sd, meta, sets, MIXED_SLOTS[sd]) for sd in MIXED_SIDES]
    pool = nmg.Pool(budget)
    for h in handles:
        pool.add(h)
    rng = np.random.default_rng(41000)
    member = rng.integers(0, len(MIXED_SIDES), size=count)
    alpha = inputs.log_uniform(1e-5, 1e-2, count, seed=41001)
    ws = np.array([select_set(set_alphas, a) for a in alpha])
    b, x = [], []
    for i in range(count):
        h, side = handles[member[i]], MIXED_SIDES[member[i]]
        u = torch.tensor(inputs.boxes_image(side - 1, 42000 + i)[None], device=dev)
        bi = h.apply_operator(0, u, torch.tensor([alpha[i]], dtype=torch.float64, device=dev), "fp64")[0]
        b.append(bi.contiguous())
        x.append(torch.empty_like(bi))
    torch.cuda.synchronize()
    # warm-up: one request per side (graph capture, coarse factors)
    for m in range(len(MIXED_SIDES)):
        i = int(np.nonzero(member == m)[0][0])
        serve_pool_requests(pool, [m], [b[i]], [x[i]], [alpha[i]], [ws[i]], np.zeros(1), precision="mixed", **kw)
    out = {"workload": f"grid side uniform over {list(MIXED_SIDES)} (n = side - 1, s = 2.5/side, levels to 15^2), "
                       f"alpha log-uniform [1e-5, 1e-2], box-image right-hand sides, Poisson arrivals, "
                       f"{count} requests per rate, budget {budget >> 20} MiB, rtol 1e-6",
           "slots": {str(sd): MIXED_SLOTS[sd] for sd in MIXED_SIDES},
           "request_mib": {str(sd): round(h.request_bytes("mixed") / 2 ** 20, 1)
                           for sd, h in zip(MIXED_SIDES, handles)}}
    for rate in rates:
        arr = inputs.poisson_arrivals(rate, count, seed=43000 + int(rate))
        arr = arr - arr[0]
        rep = serve_pool_requests(pool, member, b, x, alpha, ws, arr, precision="mixed", **kw)
        summ = rep.summary()
        ok = rep.status == 0
        summ["p99_ms_by_side"] = {str(sd): round(float(np.percentile(rep.latency_ms[(member == m) & ok], 99)), 2)
                                  for m, sd in enumerate(MIXED_SIDES) if ((member == m) & ok).any()}
        summ["mean_cycles_by_side"] = {str(sd): round(float(rep.cycles[member == m].mean()), 2)
                                       for m, sd in enumerate(MIXED_SIDES) if (member == m).any()}
        summ["converged_by_side"] = {str(sd): f"{int(((member == m) & ok).sum())}/{int((member == m).sum())}"
                                     for m, sd in enumerate(MIXED_SIDES)}
        bad = ~ok
        summ["not_converged_alpha_range"] = ([float(alpha[bad].min()), float(alpha[bad].max())]
                                             if bad.any() else None)
        out[f"poisson_{int(rate)}_per_s"] = summ
        log(f"mixed-size serving at {rate:g}/s: {summ['solves_per_s']} solves/s, p50 {summ['p50_ms']} ms, "
            f"p99 {summ['p99_ms']} ms, converged {summ['converged']}/{summ['requests']}")
    pool.close()
    if not serial:
        for h in handles:
            h.close()
        return out
    # the serial plain-FP32 solver on the first requests of the lowest rate
    rate = min(rates)
    arr = inputs.poisson_arrivals(rate, count, seed=43000 + int(rate))[:serial_count]
    arr = arr - arr[0]
    serial = [_mixed_handle(nmg, sd, meta, sets, 1) for sd in MIXED_SIDES]

    def solve_one(i):
        h1 = serial[member[i]]
        try:
            _, cyc, _, st = h1.solve(b[i][None], torch.tensor([alpha[i]], dtype=torch.float64, device=dev),
                                     weight_set=torch.tensor([int(ws[i])], dtype=torch.int32, device=dev),
                                     precision="fp32", **kw)
            return int(cyc[0]), int(st)
        except nmg.NMGError:
            return -1, -1

    for mi in range(len(serial)):  # each size's graph capture and factors before the trace
        first = next((i for i in range(len(member)) if member[i] == mi), None)
        if first is not None:
            solve_one(first)
    srep = serve_serially(solve_one, arr)
    for h1 in serial:
        h1.close()
    s_sum = srep.summary()
    s_sum["requests_of_trace"] = serial_count
    out[f"poisson_{int(rate)}_per_s"]["serial_fp32_first_requests"] = s_sum
    pool_first = out[f"poisson_{int(rate)}_per_s"]
    for h in handles:
        h.close()
    log(f"serial FP32 on the first {serial_count} requests at {rate:g}/s: p50 {s_sum['p50_ms']} ms, "
        f"p99 {s_sum['p99_ms']} ms (pool p99 {pool_first['p99_ms']} ms over {count})")
    return out


if __name__ == "__main__":
    sys.exit(main())
