"""Training-data generation of Algorithm 5 (DataGeneration) on the device,
nmg_rollout, against the oracle's data_generation: per-sample rollout
counts, V(1,0) with and without F', FP64 (1e-12) and FP32 (1e-5)."""
import pytest
import torch

import oracle as O
from paper_2603_01064_amd import inputs

pytestmark = pytest.mark.gpu
DT = torch.float64


def _rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("use_fp", [False, True])
def test_rollout_matches_oracle(use_fp):
    print(f"case rollout 63x63 k=[1,3,2,0] fprime={use_fp}", flush=True)
    from paper_2603_01064_amd import nmg
    nmg.load_library()
    dev = torch.device("cuda:0")
    n, s, L, ch, B = 63, 0.04, 3, (1, 8, 8, 1), 4
    W = [[torch.tensor(w).float().double() for w in inputs.he_normal_weights(ch, 3, 2, 7500 + 10 * l)]
         for l in range(L - 1)]
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=s, levels=L, max_batch=B, channels=ch, ksize=3))
    for l in range(L - 1):
        h.load_smoother_weights(l, 0, [w.numpy() for w in W[l]])
    H = O.build_hierarchy(n, s, L, dim=2)
    S = [O.neural_smoother(w, 2) for w in W]
    ks = [1, 3, 2, 0]
    alpha = torch.tensor([1e-2, 1e-3, 1e-4, 1e-3], dtype=DT)
    e0 = torch.tensor(inputs.iid_normal((B, n, n), 3100))
    ref_e, ref_y = O.data_generation(H, S, e0, alpha, ks, 1, 0, use_fp)
    ad = alpha.to(dev)
    e64 = e0.to(dev)
    y64 = h.rollout(e64, ad, ks, nu1=1, nu2=0, use_fprime=use_fp, precision="fp64")
    err_e, err_y = _rel(e64.cpu(), ref_e), _rel(y64.cpu(), ref_y)
    assert torch.equal(e64[3].cpu(), e0[3])  # k = 0 leaves the sample unchanged
    ref32_e, _ = O.data_generation(H, S, e0.float().double(), alpha, ks, 1, 0, use_fp)
    e32 = e0.float().to(dev)
    h.rollout(e32, ad, ks, nu1=1, nu2=0, use_fprime=use_fp, precision="fp32")
    err32 = [_rel(e32[i].cpu().double(), ref32_e[i]) for i in range(B)]
    print(f"  fp64 e {err_e:.1e} y {err_y:.1e}; fp32 per sample {['%.1e' % v for v in err32]}", flush=True)
    assert err_e < 1e-12 and err_y < 1e-12
    assert max(err32) < 1e-5
    h.close()


def test_rollout_rejects_bad_counts():
    print("case rollout bad counts", flush=True)
    from paper_2603_01064_amd import nmg
    nmg.load_library()
    dev = torch.device("cuda:0")
    h = nmg.setup_hierarchy(nmg.Problem(n=15, s=0.05, levels=2, max_batch=2, channels=(1, 4, 4, 1), ksize=3))
    h.set_jacobi_smoother(0, 0.1)
    e = torch.zeros(2, 15, 15, dtype=torch.float32, device=dev)
    alpha = torch.full((2,), 1e-2, dtype=DT, device=dev)
    with pytest.raises(nmg.NMGError):
        h.rollout(e, alpha, [1, -1])
    with pytest.raises(nmg.NMGError):
        h.rollout(e, alpha, [65, 1])
    h.close()
