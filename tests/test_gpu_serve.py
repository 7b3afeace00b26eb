"""Continuous batching: requests join and leave the batch between outer
iterations.  Every served request must give bit-identically the iterate and
cycle count of solving it alone (each right-hand side is an independent solve,
Sec. 2.3), whatever requests shared its iterations."""
import math
import os

import numpy as np
import pytest
import torch

from paper_2603_01064_amd import inputs

pytestmark = pytest.mark.gpu
DT = torch.float64
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2603_01064_amd", "weights", "grid255_s0.01.npz")


def _setup(max_batch):
    from paper_2603_01064_amd import nmg
    from paper_2603_01064_amd.train_weights import load_weights
    nmg.load_library()
    meta, sets = load_weights(WEIGHTS)
    h = nmg.setup_hierarchy(nmg.Problem(n=meta["n"], s=meta["s"], levels=meta["levels"], max_batch=max_batch,
                                        channels=(1, 32, 32, 1), ksize=3, n_weight_sets=len(sets)))
    for k, ws in enumerate(sets):
        for l in range(meta["levels"] - 1):
            h.load_smoother_weights(l, k, [ws[l]])
    return nmg, h, meta


def _wsel(meta, a):
    return min(range(len(meta["alphas"])), key=lambda i: abs(math.log(meta["alphas"][i] / a)))


def test_served_requests_equal_solo_solves():
    """Ten requests through four slots (so requests are admitted while others
    iterate); each result equals its solo solve bit for bit."""
    print("case serve 10 requests through 4 slots", flush=True)
    nmg, h, meta = _setup(4)
    dev = torch.device("cuda:0")
    n = meta["n"]
    cyc = meta["cycle"]
    al = [1e-2, 1e-4, 1e-3, 1e-2, 1e-3, 1e-4, 1e-2, 1e-3, 1e-2, 1e-4]
    u = torch.tensor(np.stack([inputs.boxes_image(n, 2600 + i) for i in range(len(al))]), device=dev)
    alpha = torch.tensor(al, dtype=DT, device=dev)
    b = torch.cat([h.apply_operator(0, u[i:i + 4], alpha[i:i + 4], "fp64") for i in range(0, len(al), 4)])
    xs = torch.zeros_like(b)
    for i, a in enumerate(al):
        h.serve_submit(b[i], xs[i], a, _wsel(meta, a), rid=100 + i)
    assert h.serve_pending() == (len(al), 0)
    kw = dict(rtol=1e-6, max_cycles=200, nu1=cyc["nu1"], nu2=cyc["nu2"], use_fprime=cyc["use_fprime"],
              precision="mixed")
    results, steps = {}, 0
    while sum(h.serve_pending()) > 0:
        for r in h.serve_step(**kw):
            results[int(r.id)] = r
        steps += 1
        assert steps < 1000
    assert sorted(results) == [100 + i for i in range(len(al))]
    total_cycles = sum(r.cycles for r in results.values())
    print(f"  steps {steps}, cycles {[results[100 + i].cycles for i in range(len(al))]}", flush=True)
    assert steps < total_cycles  # iterations were shared
    for i, a in enumerate(al):
        r = results[100 + i]
        assert r.status == 0 and r.rel_residual <= 1e-6 and r.latency_ms > 0
        ws = torch.tensor([_wsel(meta, a)], dtype=torch.int32, device=dev)
        x1, c1, _, st = h.solve(b[i:i + 1], alpha[i:i + 1], weight_set=ws, **kw)
        assert st == 0 and int(c1[0]) == r.cycles
        assert torch.equal(x1[0], xs[i])
    h.close()


def test_serve_state_rules():
    print("case serve validation and state", flush=True)
    nmg, h, meta = _setup(2)
    dev = torch.device("cuda:0")
    n = meta["n"]
    b = torch.ones(n, n, dtype=DT, device=dev)
    x = torch.zeros_like(b)
    with pytest.raises(nmg.NMGError):
        h.serve_submit(b, x, -1.0)
    with pytest.raises(nmg.NMGError):
        h.serve_submit(b, x, 1e-3, weight_set=7)
    h.serve_submit(b, x, 1e-3)
    # a batch solve shares the engine: refused while requests are queued
    with pytest.raises(nmg.NMGError):
        h.solve(b[None], torch.tensor([1e-3], dtype=DT, device=dev))
    h.serve_reset()
    assert h.serve_pending() == (0, 0)
    a = torch.tensor([1e-3], dtype=DT, device=dev)
    u = torch.tensor(inputs.boxes_image(n, 2700), device=dev)[None]
    ws = torch.tensor([_wsel(meta, 1e-3)], dtype=torch.int32, device=dev)
    xs, cyc, _, st = h.solve(h.apply_operator(0, u, a, "fp64"), a, weight_set=ws, max_cycles=200,
                             use_fprime=meta["cycle"]["use_fprime"])
    assert st == 0
    h.close()
