"""BF16 MFMA smoother: checked against a BF16-rounding emulation of the same
network (tight) and against the FP64 oracle (error stated, loose bound)."""
import pytest
import torch

import oracle as O
from paper_2603_01064_amd import inputs

pytestmark = pytest.mark.gpu
DT = torch.float64


def _bf(x):
    return x.to(torch.bfloat16).to(DT)


def _emulated_smoother(W, b):
    """Same network with every operand the kernel rounds to BF16 rounded the
    same way (input b/||b||, weights, hidden activations); sums in FP64."""
    nrm = torch.sqrt((b * b).sum(dim=(1, 2)))
    z = _bf(b / nrm[:, None, None]).unsqueeze(1)
    for i, w in enumerate(W):
        z = torch.nn.functional.conv2d(z, _bf(w), padding=1)
        if i + 1 < len(W):
            z = _bf(torch.relu(z))
    return z.squeeze(1) * nrm[:, None, None]


def _rel(a, b):
    return float((a - b).norm() / b.norm())


# batch 8 at 255 leaves fewer workgroups per image than tiles, so a workgroup
# walks several tiles (the prefetch path) for both network depths
@pytest.mark.parametrize("n,ch,B", [(63, (1, 32, 32, 1), 3), (255, (1, 32, 32, 1), 8),
                                    (31, (1, 32, 32, 32, 1), 2), (255, (1, 32, 32, 32, 1), 8),
                                    (15, (1, 32, 32, 1), 1)])
def test_mfma_smoother_matches_bf16_emulation(n, ch, B):
    print(f"case mfma smoother n={n} layers={len(ch) - 1} B={B}", flush=True)
    from paper_2603_01064_amd import nmg
    dev = torch.device("cuda:0")
    levels = {255: 5, 63: 3, 31: 2, 15: 2}[n]
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=0.02, levels=levels, max_batch=B, channels=ch, ksize=3))
    W = [torch.tensor(w).float().double() for w in inputs.he_normal_weights(ch, 3, 2, 7100)]
    h.load_smoother_weights(0, 0, [w.numpy() for w in W])
    b = torch.randn(B, n, n, dtype=DT, generator=torch.Generator().manual_seed(50)) * 3.0
    b[0, :5, :] = 0.0  # zero rows next to the boundary
    got = h.apply_smoother(0, b.float().to(dev), precision="mixed").cpu().double()
    emul = _emulated_smoother(W, b.float().double())
    e_emul = _rel(got, emul)
    ref = O.neural_smoother(W, 2)(None, 0, b, None)
    e_ref = _rel(got, ref)
    print(f"  vs bf16 emulation {e_emul:.2e}   vs fp64 oracle {e_ref:.2e}", flush=True)
    assert e_emul < 2e-4
    assert e_ref < 5e-2
    # fp32 and fp64 direct paths of the same entry point
    g32 = h.apply_smoother(0, b.float().to(dev), precision="fp32").cpu().double()
    g64 = h.apply_smoother(0, b.to(dev), precision="fp64").cpu()
    assert _rel(g64, ref) < 1e-12 and _rel(g32, ref) < 1e-5
    h.close()


def test_mfma_zero_input_gives_zero():
    print("case mfma zero input", flush=True)
    from paper_2603_01064_amd import nmg
    dev = torch.device("cuda:0")
    ch = (1, 32, 32, 1)
    h = nmg.setup_hierarchy(nmg.Problem(n=31, s=0.02, levels=2, max_batch=2, channels=ch, ksize=3))
    h.load_smoother_weights(0, 0, inputs.he_normal_weights(ch, 3, 2, 7200))
    b = torch.zeros(2, 31, 31, dtype=torch.float32, device=dev)
    out = h.apply_smoother(0, b, precision="mixed")
    assert int(torch.count_nonzero(out)) == 0 and bool(torch.isfinite(out).all())
    h.close()


def test_mixed_vcycle_error_stated():
    """Mixed-precision cycle vs FP64 oracle on 63x63 with 4 levels (error stated)."""
    print("case mixed vcycle 63", flush=True)
    from paper_2603_01064_amd import nmg
    dev = torch.device("cuda:0")
    n, s, L, ch = 63, 0.04, 4, (1, 32, 32, 1)
    W = [[torch.tensor(w).float().double() for w in inputs.he_normal_weights(ch, 3, 2, 7000 + 10 * l)] for l in range(L - 1)]
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, max_batch=2, channels=ch, ksize=3))
    for l in range(L - 1):
        h.load_smoother_weights(l, 0, [w.numpy() for w in W[l]])
    H = O.build_hierarchy(n, s, L, dim=2)
    alpha = torch.tensor([1e-2, 1e-3], dtype=DT)
    y = torch.randn(2, n, n, dtype=DT, generator=torch.Generator().manual_seed(51))
    ref = O.vcycle(H, [O.neural_smoother(w, 2) for w in W], torch.zeros_like(y), y, alpha, 1, 1, True)
    ad = alpha.to(dev)
    h.prepare(ad)
    x = torch.zeros(2, n, n, dtype=torch.float32, device=dev)
    h.vcycle(y.float().to(dev), x, ad, nu1=1, nu2=1, use_fprime=True, precision="mixed")
    err = _rel(x.cpu().double(), ref)
    print(f"  mixed V(1,1)+F' vs fp64 oracle: {err:.2e}", flush=True)
    assert err < 5e-2
    h.close()


@pytest.mark.parametrize("n,L,B,ch", [(127, 3, 3, (1, 32, 32, 1)), (255, 5, 8, (1, 32, 32, 1)),
                                      (255, 4, 5, (1, 32, 32, 32, 1)), (511, 4, 2, (1, 32, 32, 1))])
def test_mixed_cycle_bf16_plane_equals_fp32_handoff(n, L, B, ch):
    """In mixed-precision cycles with F' the BF16 smoother hands the MFMA
    filter a zero-padded BF16 plane on levels above 64^2 (the filter rounds
    an FP32 input to exactly those values itself).  Two V(1,1)+F' cycles are
    compared bit for bit with the same cycles run with the FP32 handoff
    (NMG_DEBUG_FP32_HANDOFF), which the F' parity tests cover."""
    print(f"case bf16 plane handoff n={n} L={L} B={B} layers={len(ch) - 1}", flush=True)
    from paper_2603_01064_amd import nmg
    dev = torch.device("cuda:0")
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=2.56 / (n + 1), levels=L, max_batch=B, channels=ch, ksize=3))
    for l in range(L - 1):
        h.load_smoother_weights(l, 0, inputs.he_normal_weights(ch, 3, 2, 7300 + 10 * l))
    alpha = torch.tensor([1e-2, 1e-3, 1e-4] * B, dtype=DT)[:B].to(dev)
    h.prepare(alpha)
    y = torch.randn(B, n, n, dtype=torch.float32, generator=torch.Generator().manual_seed(52)).to(dev)
    outs = []
    for handoff in (0, 1):
        h.debug_option(1, handoff)
        x = torch.zeros_like(y)
        for _ in range(2):
            h.vcycle(y, x, alpha, nu1=1, nu2=1, use_fprime=True, precision="mixed")
        torch.cuda.synchronize()
        outs.append(x.cpu())
    h.close()
    assert bool(torch.isfinite(outs[0]).all()) and float(outs[0].abs().max()) > 0
    diff = int((outs[0] != outs[1]).sum())
    print(f"  differing elements: {diff} of {outs[0].numel()}", flush=True)
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("n,L", [(63, 3), (255, 5)])
def test_fprime_every_precision(n, L):
    """F'(h) = C^T (m' .* (C h C^T)) C: FP64 / FP32 against the oracle, the BF16
    MFMA form against a stage-by-stage BF16 emulation and the oracle."""
    print(f"case fprime n={n}", flush=True)
    from paper_2603_01064_amd import nmg
    dev = torch.device("cuda:0")
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=0.02, levels=L, max_batch=2, channels=(1, 32, 32, 1), ksize=3))
    x = torch.randn(2, n, n, dtype=DT, generator=torch.Generator().manual_seed(60))
    ref = O.fprime(x, 2)
    g64 = h.apply_fprime(0, x.to(dev), "fp64").cpu()
    g32 = h.apply_fprime(0, x.float().to(dev), "fp32").cpu().double()
    gmx = h.apply_fprime(0, x.float().to(dev), "mixed").cpu().double()
    C = _bf(O.dct2_matrix(n))
    m = O.fprime_mask(n, 2)
    t = (_bf(x.float().double()) @ C.T).transpose(1, 2)
    u = (_bf(t) @ C.T).transpose(1, 2) * m
    v = (_bf(u) @ C).transpose(1, 2)
    emul = (_bf(v) @ C).transpose(1, 2)
    e64, e32, ee, er = _rel(g64, ref), _rel(g32, ref), _rel(gmx, emul), _rel(gmx, ref)
    print(f"  fp64 {e64:.1e} fp32 {e32:.1e} mixed-vs-emulation {ee:.1e} mixed-vs-oracle {er:.1e}", flush=True)
    assert e64 < 1e-12 and e32 < 1e-5 and ee < 1e-3 and er < 3e-2
    h.close()


@pytest.mark.parametrize("n", [127, 511, 1023, 2047])
def test_fprime_bf16_large_grids(n):
    """The BF16 F' at the level sizes the mixed-size serving pool and the
    large solve run (127^2 .. 2047^2; four batched MFMA passes): against its
    stage-by-stage BF16 emulation (tight) and the FP64 oracle (stated)."""
    print(f"case fprime bf16 n={n}", flush=True)
    from paper_2603_01064_amd import nmg
    dev = torch.device("cuda:0")
    # Only level 0's F' is applied; the depth keeps the coarsest grid within
    # the eigenbasis coarse solve's limit (511^2).
    levels = 2 if n <= 1023 else 3
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=2.56 / (n + 1), levels=levels, max_batch=1,
                                        channels=(1, 32, 32, 1), ksize=3))
    x = torch.randn(1, n, n, dtype=DT, generator=torch.Generator().manual_seed(61)).float().double()
    gmx = h.apply_fprime(0, x.float().to(dev), "mixed").cpu().double()
    C = _bf(O.dct2_matrix(n))
    m = O.fprime_mask(n, 2)
    t = (_bf(x) @ C.T).transpose(1, 2)
    u = (_bf(t) @ C.T).transpose(1, 2) * m
    v = (_bf(u) @ C).transpose(1, 2)
    emul = (_bf(v) @ C).transpose(1, 2)
    ref = O.fprime(x, 2)
    ee, er = _rel(gmx, emul), _rel(gmx, ref)
    print(f"  mixed-vs-emulation {ee:.1e} mixed-vs-oracle {er:.1e}", flush=True)
    assert ee < 1e-3 and er < 3e-2
    h.close()


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_solve_fp32_and_mixed_reach_tolerance(prec):
    """Damped-Jacobi cycle (no learned weights) on 31x31: the plain FP32 and
    the mixed refinement solves reach 1e-6 and agree with a dense solve."""
    print(f"case solve {prec} to 1e-6", flush=True)
    import numpy as np
    from paper_2603_01064_amd import nmg
    dev = torch.device("cuda:0")
    n, s, L, av = 31, 0.04, 3, 1e-1
    H = O.build_hierarchy(n, s, L, dim=2)
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, max_batch=2, channels=(1, 4, 4, 1), ksize=3))
    for l in range(L - 1):
        A = O.dense_operator(H, l, av)
        d = torch.diagonal(A)
        h.set_jacobi_smoother(l, 1.0 / float(torch.linalg.eigvals(A / d[:, None]).abs().max()))
    u = torch.tensor(np.stack([inputs.boxes_image(n, 2100 + i) for i in range(2)]))
    alpha = torch.full((2,), av, dtype=DT)
    y = O.apply_operator(H, 0, u, alpha)
    x, cyc, hist, st = h.solve(y.to(dev), alpha.to(dev), rtol=1e-6, max_cycles=300, precision=prec, history=True)
    assert st == 0, (cyc, hist[:, -3:])
    dense = torch.linalg.solve(O.dense_operator(H, 0, av), y.reshape(2, -1).T).T.reshape(y.shape)
    err = _rel(x.cpu(), dense)
    print(f"  cycles {list(cyc)} error vs dense {err:.2e}", flush=True)
    assert err < 1e-4
    h.close()
