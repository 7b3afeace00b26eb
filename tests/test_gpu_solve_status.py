"""Per right-hand-side outcome of nmg_solve (status, final FP64 residual,
cycles) and the divergence guard: a right-hand side whose smoother does not
fit its operator is retired on its own, flagged by index, while the others
of the same batch converge exactly as when solved alone.  Also the
forward-only loss (nmg_loss_forward) against the fused loss-and-adjoint
call."""
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


def test_divergent_rhs_is_flagged_and_the_others_finish():
    print("case divergence guard 255x255 batch 4 (one set amplified)", flush=True)
    from paper_2603_01064_amd import nmg
    from paper_2603_01064_amd.train_weights import load_weights
    nmg.load_library()
    meta, sets = load_weights(WEIGHTS)
    n, s, L = meta["n"], meta["s"], meta["levels"]
    cyc = meta["cycle"]
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, max_batch=4, channels=(1, 32, 32, 1), ksize=3,
                                        n_weight_sets=2))
    good = sets[0]  # trained for alpha 1e-2
    for l in range(L - 1):
        h.load_smoother_weights(l, 0, [good[l]])
        # every layer times 3: the bias-free ReLU network's output grows 27x,
        # so the correction overshoots and the residual grows every cycle
        h.load_smoother_weights(l, 1, [3.0 * np.asarray(good[l], dtype=np.float32)])
    dev = torch.device("cuda:0")
    alpha = torch.full((4,), 1e-2, dtype=DT, device=dev)
    u = torch.tensor(np.stack([inputs.boxes_image(n, 2300 + i) for i in range(4)]), device=dev)
    b = h.apply_operator(0, u, alpha, "fp64")
    ws = torch.tensor([0, 1, 0, 0], dtype=torch.int32, device=dev)
    kw = dict(rtol=1e-6, max_cycles=60, nu1=cyc["nu1"], nu2=cyc["nu2"], use_fprime=cyc["use_fprime"],
              precision="mixed")
    x, cycles, hist, st = h.solve(b, alpha, weight_set=ws, history=True, **kw)
    stats = h.last_stats
    print(f"  status {list(stats['status'])} cycles {list(stats['cycles'])} "
          f"rel residual {['%.2e' % v for v in stats['rel_residual']]}", flush=True)
    assert st == nmg.NMG_NOT_CONVERGED
    assert list(stats["status"]) == [nmg.NMG_OK, nmg.NMG_DIVERGED, nmg.NMG_OK, nmg.NMG_OK]
    # flagged within a few cycles, at the guard
    assert stats["cycles"][1] <= 10
    assert stats["rel_residual"][1] > 1e6
    assert hist[1, stats["cycles"][1]] > 1e6
    # final FP64 residuals reported per right-hand side match the returned iterates
    r = b - h.apply_operator(0, x, alpha, "fp64")
    rel = (r.flatten(1).norm(dim=1) / b.flatten(1).norm(dim=1)).cpu().numpy()
    for i in (0, 2, 3):
        assert stats["rel_residual"][i] <= 1e-6
        assert abs(rel[i] - stats["rel_residual"][i]) <= 1e-3 * stats["rel_residual"][i] + 1e-15
        assert stats["done_ms"][i] > 0
    # the others are exactly their solo solves
    for i in (0, 2, 3):
        xs, cs, _, ss = h.solve(b[i:i + 1], alpha[i:i + 1], weight_set=ws[i:i + 1], **kw)
        assert ss == 0 and int(cs[0]) == int(cycles[i])
        assert torch.equal(xs[0], x[i])
    h.close()


def test_solve_stats_for_max_cycles():
    """A right-hand side stopped by max_cycles reports NMG_NOT_CONVERGED with
    the residual of the iterate it returns."""
    print("case solve stats at max_cycles", flush=True)
    from paper_2603_01064_amd import nmg
    nmg.load_library()
    dev = torch.device("cuda:0")
    n, L = 31, 3
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=0.04, levels=L, max_batch=2, channels=(1, 4, 4, 1), ksize=3))
    for l in range(L - 1):
        h.set_jacobi_smoother(l, 0.05)
    alpha = torch.tensor([1e-1, 1e-1], dtype=DT, device=dev)
    u = torch.tensor(np.stack([inputs.boxes_image(n, 2400 + i) for i in range(2)]), device=dev)
    b = h.apply_operator(0, u, alpha, "fp64")
    x, cycles, _, st = h.solve(b, alpha, rtol=1e-12, max_cycles=3, precision="fp64")
    stats = h.last_stats
    assert st == nmg.NMG_NOT_CONVERGED
    assert list(stats["status"]) == [nmg.NMG_NOT_CONVERGED] * 2 and list(stats["cycles"]) == [3, 3]
    r = b - h.apply_operator(0, x, alpha, "fp64")
    rel = (r.flatten(1).norm(dim=1) / b.flatten(1).norm(dim=1)).cpu().numpy()
    assert np.allclose(rel, stats["rel_residual"], rtol=1e-9, atol=0)
    h.close()


@pytest.mark.parametrize("mask,prec", [("ramp", "fp64"), ("band", "fp32"), ("cycle", "fp64"), ("ramp", "mixed")])
def test_loss_forward_equals_loss_grad(mask, prec):
    """nmg_loss_forward gives the losses nmg_loss_grad reports for the same
    inputs (same kernels, bit for bit) and leaves the gradients alone."""
    print(f"case loss forward {mask} {prec}", flush=True)
    from paper_2603_01064_amd import nmg
    nmg.load_library()
    dev = torch.device("cuda:0")
    n, L, ch = 31, 4, (1, 32, 32, 1)
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=0.05, levels=L, max_batch=3, channels=ch, ksize=3))
    for l in range(L - 1):
        h.load_smoother_weights(l, 0, inputs.he_normal_weights(ch, 3, 2, 7300 + 10 * l))
    dt = DT if prec == "fp64" else torch.float32
    g = torch.Generator().manual_seed(5)
    e1 = torch.randn(3, n, n, dtype=DT, generator=g).to(dt).to(dev)
    e2 = torch.randn(3, n, n, dtype=DT, generator=g).to(dt).to(dev)
    alpha = torch.tensor([1e-2, 1e-3, 1e-4], dtype=DT, device=dev)
    l1 = h.loss_grad(e1, alpha, mask=mask, use_fprime=True, precision=prec)
    g1 = [h.get_gradient(l) for l in range(L - 1)]
    f2 = h.loss_forward(e2, alpha, mask=mask, use_fprime=True, precision=prec)
    g1b = [h.get_gradient(l) for l in range(L - 1)]
    assert all(np.array_equal(a, b) for a, b in zip(g1, g1b))
    f1 = h.loss_forward(e1, alpha, mask=mask, use_fprime=True, precision=prec)
    assert np.array_equal(f1, l1), (f1, l1)
    l2 = h.loss_grad(e2, alpha, mask=mask, use_fprime=True, precision=prec)
    assert np.array_equal(f2, l2)
    assert not np.array_equal(f1, f2)
    h.close()


def test_autograd_skips_the_adjoint_without_grad():
    """Under torch.no_grad the autograd wrapper evaluates the losses only."""
    print("case autograd forward only", flush=True)
    from paper_2603_01064_amd import autograd, nmg
    nmg.load_library()
    dev = torch.device("cuda:0")
    n, L, ch = 31, 3, (1, 8, 8, 1)
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=0.05, levels=L, max_batch=2, channels=ch, ksize=3))
    W = [torch.tensor(np.concatenate([w.reshape(-1) for w in inputs.he_normal_weights(ch, 3, 2, 7400 + 10 * l)]),
                      dtype=torch.float32) for l in range(L - 1)]
    for l in range(L - 1):
        h.load_smoother_weights(l, 0, [W[l].numpy()])
    e = torch.randn(2, n, n, dtype=DT, generator=torch.Generator().manual_seed(6)).to(dev)
    alpha = torch.tensor([1e-2, 1e-3], dtype=DT, device=dev)
    h.loss_grad(e, alpha, mask="ramp", precision="fp64")
    g0 = [h.get_gradient(l) for l in range(L - 1)]
    with torch.no_grad():
        out = autograd.levelwise_loss(h, W, 2.0 * e, alpha, mask="ramp", precision="fp64")
    assert all(np.array_equal(a, h.get_gradient(l)) for l, a in enumerate(g0))
    ref = h.loss_forward(2.0 * e, alpha, mask="ramp", precision="fp64")
    assert np.array_equal(out.numpy(), ref)
    h.close()
