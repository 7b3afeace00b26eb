"""The autograd wrapper over the hand-written adjoint (pattern: custom
torch.autograd.Function): gradients through ``backward`` equal the FP64
oracle's autograd gradients of the same level-wise losses (Sec. 3.3 eq.
loss_3, gradient of each level's loss w.r.t. its own smoother), scaled by
arbitrary incoming loss weights; and a torch optimiser can train through it."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2603_01064_amd import inputs

pytestmark = pytest.mark.gpu
DT = torch.float64


def _flat32(ws):
    return torch.cat([w.reshape(-1) for w in ws]).float().double()


def test_backward_equals_oracle_autograd_fp64():
    print("case autograd wrapper fp64 31x31", flush=True)
    from paper_2603_01064_amd import nmg
    from paper_2603_01064_amd.autograd import levelwise_loss
    dev = torch.device("cuda:0")
    n, s, L, ch, B = 31, 0.04, 4, (1, 32, 32, 1), 3
    W = [[torch.tensor(w).float().double() for w in inputs.he_normal_weights(ch, 3, 2, 7400 + 10 * l)]
         for l in range(L - 1)]
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, max_batch=B, channels=ch, ksize=3))
    H = O.build_hierarchy(n, s, L, dim=2)
    e = torch.tensor(inputs.iid_normal((B, n, n), 3100))
    alpha = torch.full((B,), 1e-3, dtype=DT)
    params = [_flat32(lw).requires_grad_(True) for lw in W]
    losses = levelwise_loss(h, params, e.to(dev), alpha.to(dev), mask="ramp", precision="fp64")
    c = torch.tensor([1.0, 2.0, 0.5], dtype=DT)
    (c * losses).sum().backward()
    ref_l, ref_g = O.level_loss_grads(H, W, e, alpha, "ramp", False)
    got = losses.detach()
    for l in range(L - 1):
        assert abs(float(got[l]) - float(ref_l[l])) <= 1e-12 * abs(float(ref_l[l]))
        r = float(c[l]) * torch.cat([g.reshape(-1) for g in ref_g[l]])
        err = float((params[l].grad - r).norm() / r.norm())
        print(f"  level {l}: grad rel err {err:.2e}", flush=True)
        assert err < 1e-10
    h.close()


def test_torch_adam_trains_through_the_wrapper():
    print("case torch Adam through the wrapper fp32 63x63", flush=True)
    from paper_2603_01064_amd import nmg
    from paper_2603_01064_amd.autograd import levelwise_loss
    dev = torch.device("cuda:0")
    n, s, L, ch, B = 63, 0.02, 3, (1, 32, 32, 1), 8
    W = [[torch.tensor(w).float() for w in inputs.he_normal_weights(ch, 3, 2, 7500 + 10 * l)] for l in range(L - 1)]
    params = [torch.cat([w.reshape(-1) for w in lw]).requires_grad_(True) for lw in W]
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, max_batch=B, channels=ch, ksize=3))
    opt = torch.optim.Adam(params, lr=1e-3)
    alpha = torch.full((B,), 1e-3, dtype=DT, device=dev)
    first = last = None
    for step in range(30):
        e = torch.tensor(inputs.iid_normal((B, n, n), 3200 + step), dtype=torch.float32).to(dev)
        opt.zero_grad()
        losses = levelwise_loss(h, params, e, alpha, mask="ramp", precision="fp32")
        losses.sum().backward()
        opt.step()
        total = float(losses.sum())
        first = total if first is None else first
        last = total
    print(f"  loss {first:.4e} -> {last:.4e}", flush=True)
    assert np.isfinite(last) and last < 0.9 * first
    h.close()
