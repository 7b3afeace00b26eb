"""FNO smoother (Sec. 3.1; the appendix's network description) on the GPU
against the oracle: the smoother on every level in FP64 (1e-12) and FP32
(1e-5), V-cycles with FNO smoothers, and per-right-hand-side weight sets."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2603_01064_amd import inputs
from paper_2603_01064_amd.fno import pack_fno_weights

pytestmark = pytest.mark.gpu
DT = torch.float64


def _oracle_params(p):
    t = lambda a: torch.tensor(np.asarray(a), dtype=DT)
    return {"lift_w": t(p["lift_w"]), "lift_b": t(p["lift_b"]), "proj_w": t(p["proj_w"]), "proj_b": t(p["proj_b"]),
            "layers": [{"R": torch.complex(t(L["R_re"]), t(L["R_im"])), "W": t(L["W"]), "B": t(L["B"])}
                       for L in p["layers"]]}


def _setup(dim, n, s, L, arch, B=2, sets=1, seed=7700):
    from paper_2603_01064_amd import nmg
    nmg.load_library()
    C, NL, m, ks = arch
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, dim=dim, max_batch=B, n_weight_sets=sets, fno=arch))
    params = [[inputs.fno_params(dim, C, NL, m, ks, seed + 100 * k + 10 * l) for l in range(L - 1)]
              for k in range(sets)]
    for k in range(sets):
        for l in range(L - 1):
            flat = pack_fno_weights(params[k][l])
            assert flat.size == h.problem.weight_count()
            h.load_smoother_weights(l, k, [flat])
    H = O.build_hierarchy(n, s, L, dim=dim)
    return h, H, params


def _rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("dim,n,s,L,arch", [(2, 63, 0.04, 3, (8, 2, 8, 3)), (2, 31, 0.05, 3, (4, 3, 12, 5)),
                                            (1, 127, 0.02, 3, (6, 2, 16, 5)), (2, 63, 0.04, 3, (32, 2, 8, 5)),
                                            (2, 63, 0.04, 3, (16, 2, 6, 3)), (2, 63, 0.04, 3, (16, 1, 6, 7)),
                                            (2, 31, 0.05, 3, (16, 1, 4, 9)), (2, 63, 0.04, 3, (32, 1, 6, 3)),
                                            (2, 31, 0.05, 3, (32, 1, 4, 7)), (2, 63, 0.04, 3, (64, 1, 6, 3))])
def test_fno_smoother_every_level(dim, n, s, L, arch):
    """Mode counts clamp on the coarse levels (k_l = min(k, n_l / 2)).  Widths
    that are multiples of 16 run the LDS-tiled 2D layer kernels: 32 x 32
    tiles with 2 x 2 pixels per thread for 3 x 3, 5 x 5 and 7 x 7
    convolutions, 16 x 16 tiles otherwise (9 x 9 here); in FP32, widths 32
    and 64 with those three kernel sizes run the MFMA layer kernel (32 x 8
    tiles); the tiles are ragged at 63 and 31."""
    print(f"case FNO smoother dim={dim} n={n} arch={arch}", flush=True)
    dev = torch.device("cuda:0")
    h, H, params = _setup(dim, n, s, L, arch)
    g = torch.Generator().manual_seed(50)
    alpha = torch.tensor([1e-2, 1e-3], dtype=DT)
    for l in range(L - 1):
        nl = H.levels[l].n
        b = torch.randn((2,) + (nl,) * dim, dtype=DT, generator=g)
        b[1] *= 1e-3  # the network sees b / ||b||; h scales with ||b||
        ref = O.fno_smoother(_oracle_params(params[0][l]), dim, arch[2])(H, l, b, alpha)
        got = h.apply_smoother(l, b.to(dev), alpha.to(dev), precision="fp64").cpu()
        assert _rel(got, ref) < 1e-12, l
        b32 = b.float().double()
        ref32 = O.fno_smoother(_oracle_params(params[0][l]), dim, arch[2])(H, l, b32, alpha)
        got32 = h.apply_smoother(l, b.float().to(dev), alpha.to(dev), precision="fp32").cpu().double()
        print(f"  level {l} (n={nl}, k={O.fno_modes(nl, arch[2])}): fp32 rel err {_rel(got32, ref32):.2e}",
              flush=True)
        assert _rel(got32, ref32) < 1e-5, l
    zero = torch.zeros((1,) + (H.levels[0].n,) * dim, dtype=DT, device=dev)
    assert float(h.apply_smoother(0, zero, alpha[:1].to(dev), precision="fp64").abs().max()) == 0.0
    h.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("mixed", 3e-2)])
def test_fno_vcycle_matches_oracle(prec, tol):
    """Three V(1,1)+F' cycles with FNO smoothers on every level against the
    oracle's cycle.  The FNO runs in FP32 inside mixed-precision cycles, whose
    F' is the BF16 MFMA filter (its rounding, about 1e-3 here, sets the mixed
    tolerance)."""
    print(f"case FNO V-cycle {prec}", flush=True)
    dev = torch.device("cuda:0")
    dim, n, s, L, arch = 2, 63, 0.04, 3, (8, 2, 8, 3)
    h, H, params = _setup(dim, n, s, L, arch)
    S = [O.fno_smoother(_oracle_params(params[0][l]), dim, arch[2]) for l in range(L - 1)]
    alpha = torch.tensor([1e-2, 1e-3], dtype=DT)
    y = torch.randn(2, n, n, dtype=DT, generator=torch.Generator().manual_seed(51))
    if prec != "fp64":
        y = y.float().double()
    x = torch.zeros_like(y)
    dt = torch.float64 if prec == "fp64" else torch.float32
    xd = x.to(dt).to(dev)
    ad = alpha.to(dev)
    h.prepare(ad)
    for c in range(3):
        x = O.vcycle(H, S, x, y, alpha, 1, 1, True)
        h.vcycle(y.to(dt).to(dev), xd, ad, nu1=1, nu2=1, use_fprime=True, precision=prec)
        d = float(O.apply_operator(H, 0, xd.cpu().double() - x, alpha).norm() / y.norm())
        print(f"  cycle {c}: ||A (x - x_ref)|| / ||y|| = {d:.2e}", flush=True)
        assert d < tol
    h.close()


def test_fno_weight_sets_per_rhs():
    """Each right-hand side picks its own FNO weight set; results equal solo runs."""
    print("case FNO per-RHS weight sets", flush=True)
    dev = torch.device("cuda:0")
    dim, n, s, L, arch = 2, 31, 0.05, 3, (4, 2, 6, 3)
    h, H, params = _setup(dim, n, s, L, arch, B=2, sets=2)
    b = torch.randn(2, n, n, dtype=DT, generator=torch.Generator().manual_seed(52)).to(dev)
    alpha = torch.tensor([1e-2, 1e-2], dtype=DT, device=dev)
    ws = torch.tensor([1, 0], dtype=torch.int32, device=dev)
    both = h.apply_smoother(0, b, alpha, weight_set=ws, precision="fp64")
    for i in range(2):
        solo = h.apply_smoother(0, b[i:i + 1], alpha[i:i + 1], weight_set=ws[i:i + 1], precision="fp64")
        assert torch.equal(solo[0], both[i])
        ref = O.fno_smoother(_oracle_params(params[int(ws[i])][0]), dim, arch[2])(H, 0, b[i:i + 1].cpu(),
                                                                                   alpha[i:i + 1].cpu())
        assert _rel(both[i:i + 1].cpu(), ref) < 1e-12
    h.close()


def test_fno_weight_sets_per_rhs_fp32_mfma():
    """Per-right-hand-side weight sets on the FP32 MFMA layer kernel (width
    32): each image takes its set's copy of the convolution weights; batched
    results equal solo runs bit for bit and match the oracle to 1e-5."""
    print("case FNO per-RHS weight sets, FP32 MFMA layer kernel", flush=True)
    dev = torch.device("cuda:0")
    dim, n, s, L, arch = 2, 63, 0.04, 3, (32, 2, 6, 5)
    h, H, params = _setup(dim, n, s, L, arch, B=3, sets=2, seed=7900)
    b = torch.randn(3, n, n, dtype=DT, generator=torch.Generator().manual_seed(53)).float().double()
    alpha = torch.tensor([1e-2, 1e-3, 1e-2], dtype=DT)
    ws = torch.tensor([1, 0, 1], dtype=torch.int32, device=dev)
    both = h.apply_smoother(0, b.float().to(dev), alpha.to(dev), weight_set=ws, precision="fp32")
    for i in range(3):
        solo = h.apply_smoother(0, b[i:i + 1].float().to(dev), alpha[i:i + 1].to(dev), weight_set=ws[i:i + 1],
                                precision="fp32")
        assert torch.equal(solo[0], both[i])
        ref = O.fno_smoother(_oracle_params(params[int(ws[i])][0]), dim, arch[2])(H, 0, b[i:i + 1], alpha[i:i + 1])
        err = _rel(both[i:i + 1].cpu().double(), ref)
        print(f"  rhs {i} set {int(ws[i])}: fp32 rel err {err:.2e}", flush=True)
        assert err < 1e-5
    h.close()


# --------------------------------------------------------------------------
# Training: the hand-written FNO adjoint of the level-wise loss
# --------------------------------------------------------------------------


def _flat_grads(g):
    parts = [g["lift_w"], g["lift_b"]]
    for Ly in g["layers"]:
        parts += [Ly["R_re"], Ly["R_im"], Ly["W"], Ly["B"]]
    parts += [g["proj_w"], g["proj_b"].reshape(1)]
    return torch.cat([t.reshape(-1) for t in parts])


def _oracle_real(p):
    t = lambda a: torch.tensor(np.asarray(a), dtype=DT)
    return {"lift_w": t(p["lift_w"]), "lift_b": t(p["lift_b"]), "proj_w": t(p["proj_w"]), "proj_b": t(p["proj_b"]),
            "layers": [{k: t(L[k]) for k in ("R_re", "R_im", "W", "B")} for L in p["layers"]]}


@pytest.mark.parametrize("dim,n,s,L,arch,use_fp", [(2, 31, 0.05, 3, (4, 2, 6, 3), True),
                                                   (2, 31, 0.05, 3, (4, 1, 10, 3), False),
                                                   (1, 63, 0.03, 3, (4, 2, 8, 5), True)])
def test_fno_loss_gradient_matches_oracle(dim, n, s, L, arch, use_fp):
    """FP64 level losses 1e-12 and every level's gradient 1e-10 against the
    oracle's autograd (modes clamp on the 15-point level in the second case);
    FP32 within 1e-4."""
    print(f"case FNO loss gradient dim={dim} n={n} arch={arch}", flush=True)
    dev = torch.device("cuda:0")
    h, H, params = _setup(dim, n, s, L, arch, B=2)
    e = torch.tensor(inputs.iid_normal((2,) + (n,) * dim, 3100))
    alpha = torch.tensor([1e-2, 1e-3], dtype=DT)
    ref_l, ref_g = O.fno_level_loss_grads(H, [_oracle_real(p) for p in params[0]], e, alpha, arch[2], "ramp", use_fp)
    got = h.loss_grad(e.to(dev), alpha.to(dev), mask="ramp", use_fprime=use_fp, precision="fp64")
    for l in range(L - 1):
        assert abs(got[l] - float(ref_l[l])) <= 1e-12 * abs(float(ref_l[l]))
        g = torch.tensor(h.get_gradient(l))
        r = _flat_grads(ref_g[l])
        err = float((g - r).norm() / r.norm())
        print(f"  level {l}: loss {got[l]:.6e} grad rel err {err:.2e}", flush=True)
        assert err < 1e-10
    got32 = h.loss_grad(e.float().to(dev), alpha.to(dev), mask="ramp", use_fprime=use_fp, precision="fp32")
    for l in range(L - 1):
        g = torch.tensor(h.get_gradient(l))
        r = _flat_grads(ref_g[l])
        assert float((g - r).norm() / r.norm()) < 1e-4
        assert abs(got32[l] - float(ref_l[l])) <= 1e-4 * abs(float(ref_l[l]))
    h.close()


def test_fno_training_reduces_the_loss():
    print("case FNO training 20 steps", flush=True)
    dev = torch.device("cuda:0")
    h, H, params = _setup(2, 31, 0.05, 3, (8, 2, 6, 3), B=8)
    e = torch.tensor(inputs.iid_normal((8, 31, 31), 3101)).float().to(dev)
    alpha = torch.full((8,), 1e-2, dtype=DT, device=dev)
    first = h.train_step(e, alpha, mask="ramp", use_fprime=True, precision="fp32", lr=1e-3)
    for _ in range(20):
        last = h.train_step(e, alpha, mask="ramp", use_fprime=True, precision="fp32", lr=1e-3)
    print(f"  losses {first} -> {last}", flush=True)
    assert float(np.sum(last)) < float(np.sum(first))
    h.close()


@pytest.mark.parametrize("n", [127, 255])
def test_fno_at_the_benchmarked_architecture(n):
    """The network the benchmark times (the appendix's h = 1/256 network:
    C = 64, 5 Fourier layers, k = 32, 5 x 5 convolution) at 127^2 and at the
    timed 255^2, FP32 against the oracle on the finest level."""
    print(f"case FNO C=64 5 layers k=32 ks=5 at {n}x{n}", flush=True)
    dev = torch.device("cuda:0")
    arch = (64, 5, 32, 5)
    h, H, params = _setup(2, n, 0.01, 2, arch, B=1, seed=47000)
    b = torch.randn(1, n, n, dtype=DT, generator=torch.Generator().manual_seed(52)).float().double()
    alpha = torch.tensor([1e-3], dtype=DT)
    ref = O.fno_smoother(_oracle_params(params[0][0]), 2, arch[2])(H, 0, b, alpha)
    got = h.apply_smoother(0, b.float().to(dev), alpha.to(dev), precision="fp32").cpu().double()
    err = _rel(got, ref)
    print(f"  fp32 rel err {err:.2e}", flush=True)
    assert err < 1e-5
    h.close()
