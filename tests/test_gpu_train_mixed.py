"""Mixed-precision training (BF16 network operands, FP32 sums, FP32 loss
transforms): the library's level-wise losses and their adjoint against a
BF16-rounding emulation of the same network in FP64 (tight; the adjoint
differentiates the roundings as the identity) and against the FP64 oracle
(error stated, loose bound).  The training forward runs the BF16 MFMA
smoother; the backward recomputes the same BF16-rounded activations."""
import pytest
import torch
import torch.nn.functional as F

import oracle as O
from paper_2603_01064_amd import inputs

pytestmark = pytest.mark.gpu
DT = torch.float64


def _bf_st(x):
    """BF16 rounding with an identity derivative (straight-through)."""
    return x + (x.to(torch.bfloat16).to(DT) - x).detach()


def _emulated(weights):
    def apply(H, l, b, alpha):
        nrm = O.batch_norm2(b)
        safe = torch.where(nrm > 0, nrm, torch.ones_like(nrm))
        z = _bf_st(b / safe[:, None, None]).unsqueeze(1)
        for i, w in enumerate(weights):
            z = F.conv2d(z, _bf_st(w), padding=w.shape[-1] // 2)
            if i + 1 < len(weights):
                z = _bf_st(torch.relu(z))
        return z.squeeze(1) * nrm[:, None, None]
    return apply


def _flat(ws):
    return torch.cat([w.reshape(-1) for w in ws])


@pytest.mark.parametrize("n,L,mask,use_fp,ch", [(31, 4, "ramp", True, (1, 32, 32, 1)),
                                                 (63, 3, "band", False, (1, 32, 32, 1)),
                                                 (63, 4, "ramp", True, (1, 32, 32, 1)),
                                                 (31, 3, "ramp", True, (1, 32, 32, 32, 1))])
def test_mixed_loss_and_gradient(n, L, mask, use_fp, ch):
    """The backward runs on MFMA with BF16 activations and BF16 deltas, so the
    gradient carries their rounding on top of the emulation's (a few 1e-3)."""
    print(f"case mixed training {n}x{n} L={L} mask={mask} fprime={use_fp} layers={len(ch) - 1}", flush=True)
    from paper_2603_01064_amd import nmg
    nmg.load_library()
    dev = torch.device("cuda:0")
    B, s = 4, 0.04
    W = [[torch.tensor(w).float().double() for w in inputs.he_normal_weights(ch, 3, 2, 7600 + 10 * l)]
         for l in range(L - 1)]
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, max_batch=B, channels=ch, ksize=3))
    for l in range(L - 1):
        h.load_smoother_weights(l, 0, [w.numpy() for w in W[l]])
    H = O.build_hierarchy(n, s, L, dim=2)
    e = torch.tensor(inputs.iid_normal((B, n, n), 3200)).float().double()
    alpha = torch.tensor([1e-2, 1e-3, 1e-3, 1e-4], dtype=DT)
    got = h.loss_grad(e.float().to(dev), alpha.to(dev), mask=mask, use_fprime=use_fp, precision="mixed")
    gg = [torch.tensor(h.get_gradient(l)) for l in range(L - 1)]
    # BF16 emulation (FP64 sums) with straight-through rounding
    ws = [[w.clone().requires_grad_(True) for w in lw] for lw in W]
    em_losses = O.level_losses(H, ws, e, alpha, mask, use_fp, make_smoother=_emulated)
    sum(em_losses).backward()
    em_l = torch.stack([x.detach() for x in em_losses])
    em_g = [_flat([w.grad for w in lw]) for lw in ws]
    ref_l, ref_g = O.level_loss_grads(H, W, e, alpha, mask, use_fp)
    for l in range(L - 1):
        le = abs(got[l] - float(em_l[l])) / float(em_l[l])
        lr = abs(got[l] - float(ref_l[l])) / float(ref_l[l])
        ge = float((gg[l] - em_g[l]).norm() / em_g[l].norm())
        gr = float((gg[l] - _flat(ref_g[l])).norm() / _flat(ref_g[l]).norm())
        ger = float((em_g[l] - _flat(ref_g[l])).norm() / _flat(ref_g[l]).norm())
        print(f"  level {l}: loss vs BF16 emulation {le:.1e}, vs FP64 oracle {lr:.1e}; gradient vs emulation "
              f"{ge:.1e}, vs FP64 oracle {gr:.1e} (emulation vs oracle {ger:.1e})", flush=True)
        assert le < 2e-3 and lr < 5e-2
        assert ge < 2e-2 and gr < 2e-1
    h.close()


@pytest.mark.parametrize("use_fp", [True, False])
def test_mixed_cycle_loss_and_gradient(use_fp):
    """The combined loss eq. loss_1 in mixed precision (every level's network
    backward on MFMA, including the gradient at its input): the loss and the
    joint gradient against the same cycle with the BF16-rounding emulation of
    each smoother (FP64 sums, straight-through roundings), and against the
    FP64 oracle (stated, loose)."""
    print(f"case mixed cycle loss 31x31 L=3 fprime={use_fp}", flush=True)
    from paper_2603_01064_amd import nmg
    nmg.load_library()
    dev = torch.device("cuda:0")
    n, L, ch, B, s = 31, 3, (1, 32, 32, 1), 4, 0.04
    W = [[torch.tensor(w).float().double() for w in inputs.he_normal_weights(ch, 3, 2, 7700 + 10 * l)]
         for l in range(L - 1)]
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, max_batch=B, channels=ch, ksize=3))
    for l in range(L - 1):
        h.load_smoother_weights(l, 0, [w.numpy() for w in W[l]])
    H = O.build_hierarchy(n, s, L, dim=2)
    e = torch.tensor(inputs.iid_normal((B, n, n), 3300)).float().double()
    alpha = torch.tensor([1e-2, 1e-3, 1e-3, 1e-4], dtype=DT)
    got = h.loss_grad(e.float().to(dev), alpha.to(dev), mask="cycle", use_fprime=use_fp, precision="mixed")
    gg = [torch.tensor(h.get_gradient(l)) for l in range(L - 1)]
    ws = [[w.clone().requires_grad_(True) for w in lw] for lw in W]
    y = O.apply_operator(H, 0, e, alpha)
    x = O.vcycle(H, [_emulated(lw) for lw in ws], torch.zeros_like(e), y, alpha, 1, 0, use_fp)
    em_loss = ((e - x) ** 2).sum() / B
    em_loss.backward()
    em_g = [_flat([w.grad for w in lw]) for lw in ws]
    ref_loss, ref_g = O.cycle_loss_grads(H, W, e, alpha, use_fp)
    le = abs(got[0] - float(em_loss)) / float(em_loss)
    lr = abs(got[0] - float(ref_loss)) / float(ref_loss)
    print(f"  loss vs emulation {le:.1e}, vs FP64 oracle {lr:.1e}", flush=True)
    assert le < 2e-3 and lr < 5e-2
    for l in range(L - 1):
        ge = float((gg[l] - em_g[l]).norm() / em_g[l].norm())
        gr = float((gg[l] - _flat(ref_g[l])).norm() / _flat(ref_g[l]).norm())
        print(f"  level {l}: gradient vs emulation {ge:.1e}, vs FP64 oracle {gr:.1e}", flush=True)
        assert ge < 2e-2 and gr < 2e-1
    h.close()
